// Newton-Raphson update of the self-consistent potential (Sec. III-A item 3:
// the converged potential is obtained by Newton-Raphson iteration).
//
// The loop's fixed point U_out(U) = U is the root of
//     G(U) = A U - kappa (n(U) - N_D),   A = -Lap_h,  kappa = 1 / (h^3 eps0 eps_r),
// on the Poisson grid (n and N_D on the atoms' nodes).  Its Jacobian is
// J = A - kappa chi with chi = dn/dU, taken here from first-order
// perturbation theory over K states psi_i of the step (real H):
//     chi v = sum_p c_p rho_p (rho_p . v) + c_d d (d . v),
// one term per state pair p = (i, k), i <= k, with the pair density
// rho_p(atom) = sum_alpha psi_i psi_k, c_p = 2 g_ii (i = k) or 4 g_ik,
// g_ik = (f_i - f_k) / (E_i - E_k) (the slope at the mean level for levels
// closer than 1e-5 kT), and the Fermi level's shift under neutrality
// d = sum_i f'_i rho_ii, c_d = -2 / sum_i f'_i.  chi is symmetric negative
// semi-definite, so J is symmetric positive definite: J x = G is solved by
// conjugate gradients with the Jacobi preconditioner diag(J), and the step
// is -x.  Successive
// steps are combined by Anderson mixing (type II) over the last m steps.
//
// Data: the pair densities R [pairs][atoms] FP64 (pairs whose coefficient
// is below 1e-14 of the largest are dropped); grid vectors FP64.  Per CG
// iteration the pair densities are read twice (a_p = rho_p . v, then
// sum_p a_p rho_p): HBM-bound at 16 bytes per pair and atom.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

#include "scf.h"
#include "tbh_internal.h"

namespace tbh {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ double warp_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// block sum of one double (256 threads); valid in thread 0
__device__ double block_sum(double v) {
    __shared__ double sh[TPB / 64];
    v = warp_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    __syncthreads();
    return r;
}

__device__ double sum_part(const double* part, int64_t n) {
    double v = 0.0;
    for (int64_t b = threadIdx.x; b < n; b += TPB) v += part[b];
    return block_sum(v);
}

#define NGRID_LOOP(i, n) \
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < (n); i += int64_t(gridDim.x) * TPB)

int64_t blocks_for(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>((n + TPB - 1) / TPB, 4096)); }

// scalar slots of the preconditioned CG state
enum { NC_RZ = 0, NC_ALPHA = 1, NC_BETA = 2, NC_DONE = 3, NC_BB = 4, NC_ITERS = 5, NC_REL = 6, NC_NS = 8 };

// R[p][j] = sum_alpha y_si(j, alpha) y_sk(j, alpha) / (|y_si| |y_sk|)
__global__ void k_pair_density(const double* __restrict__ Y, int64_t ns, int n_o, int64_t n_atoms,
                               const int2* __restrict__ pairs, const int* __restrict__ sel,
                               const double* __restrict__ inv_norm, double* __restrict__ R) {
    const int p = blockIdx.y;
    const int2 ik = pairs[p];
    const double* yi = Y + int64_t(sel[ik.x]) * ns;
    const double* yk = Y + int64_t(sel[ik.y]) * ns;
    const double w = inv_norm[ik.x] * inv_norm[ik.y];
    double* out = R + int64_t(p) * n_atoms;
    NGRID_LOOP(j, n_atoms) {
        double s = 0.0;
        for (int a = 0; a < n_o; ++a) s += yi[j * n_o + a] * yk[j * n_o + a];
        out[j] = s * w;
    }
}

// d_j = sum_i f'_i rho_ii(j); chi_jj = sum_p c_p rho_p(j)^2 + c_d d_j^2; the
// preconditioner 1 / J_jj = 1 / (6 / h^2 - kappa chi_jj) at the atom's node
__global__ void k_newton_diag(int64_t n_atoms, const double* __restrict__ R, const double* __restrict__ coef,
                              int npairs, const int* __restrict__ diag_pair, const double* __restrict__ fp, int K,
                              double cd, double kappa, double a_diag, const int64_t* __restrict__ node,
                              double* __restrict__ d, double* __restrict__ minv) {
    NGRID_LOOP(j, n_atoms) {
        double dj = 0.0;
        for (int i = 0; i < K; ++i) dj += fp[i] * R[int64_t(diag_pair[i]) * n_atoms + j];
        double cjj = cd * dj * dj;
        for (int p = 0; p < npairs; ++p) {
            const double r = R[int64_t(p) * n_atoms + j];
            cjj += coef[p] * r * r;
        }
        d[j] = dj;
        minv[node[j]] = 1.0 / (a_diag - kappa * cjj);
    }
}

__global__ void k_fill(int64_t n, double v, double* x) {
    NGRID_LOOP(i, n) x[i] = v;
}

// y = A x + b (b may be null)
__global__ void k_apply_a(int nx, int ny, int nz, double inv_h2, const double* __restrict__ x,
                          const double* __restrict__ b, double* __restrict__ y, const double* done) {
    if (done && *done != 0.0) return;
    const int64_t n = int64_t(nx) * ny * nz;
    NGRID_LOOP(i, n) {
        const int xi = int(i % nx);
        const int yi = int((i / nx) % ny);
        const int zi = int(i / (int64_t(nx) * ny));
        const int64_t row = i - xi, plane = i - xi - int64_t(yi) * nx;
        double s = x[row + (xi + 1 == nx ? 0 : xi + 1)] + x[row + (xi == 0 ? nx - 1 : xi - 1)];
        s += x[plane + int64_t(yi + 1 == ny ? 0 : yi + 1) * nx + xi] +
             x[plane + int64_t(yi == 0 ? ny - 1 : yi - 1) * nx + xi];
        if (zi + 1 < nz) s += x[i + int64_t(nx) * ny];
        if (zi > 0) s += x[i - int64_t(nx) * ny];
        y[i] = (6.0 * x[i] - s) * inv_h2 + (b ? b[i] : 0.0);
    }
}

// va[j] = v[node[j]]: the grid vector on the atoms
__global__ void k_gather_nodes(int64_t n_atoms, const int64_t* __restrict__ node, const double* __restrict__ v,
                               double* __restrict__ va, const double* done) {
    if (*done != 0.0) return;
    NGRID_LOOP(j, n_atoms) va[j] = v[node[j]];
}

// a_p = c_p rho_p . va (blocks 0..npairs-1), a_npairs = c_d d . va (last block)
__global__ void k_pair_dot(int64_t n_atoms, const double* __restrict__ R, int npairs,
                           const double* __restrict__ va, const double* __restrict__ d,
                           const double* __restrict__ coef, double cd, double* __restrict__ a, const double* done) {
    if (*done != 0.0) return;
    const int p = blockIdx.x;
    const double* w = p < npairs ? R + int64_t(p) * n_atoms : d;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < n_atoms; j += TPB) s += w[j] * va[j];
    s = block_sum(s);
    if (threadIdx.x == 0) a[p] = s * (p < npairs ? coef[p] : cd);
}

// partial sums over the pairs of chunk blockIdx.y: tpart[chunk][j] = sum_{p in chunk} a_p rho_p(j)
__global__ void k_chi_partial(int64_t n_atoms, const double* __restrict__ R, int npairs, int per_chunk,
                              const double* __restrict__ a, double* __restrict__ tpart, const double* done) {
    if (*done != 0.0) return;
    const int p0 = blockIdx.y * per_chunk;
    const int p1 = p0 + per_chunk < npairs ? p0 + per_chunk : npairs;
    NGRID_LOOP(j, n_atoms) {
        double t = 0.0;
        for (int p = p0; p < p1; ++p) t += a[p] * R[int64_t(p) * n_atoms + j];
        tpart[int64_t(blockIdx.y) * n_atoms + j] = t;
    }
}

// Av[node_j] -= kappa (sum over chunks, in order, + a_d d_j)
__global__ void k_chi_apply(int64_t n_atoms, int nchunk, const double* __restrict__ tpart, int npairs,
                            const double* __restrict__ a, const double* __restrict__ d,
                            const int64_t* __restrict__ node, double kappa, double* __restrict__ Av,
                            const double* done) {
    if (*done != 0.0) return;
    NGRID_LOOP(j, n_atoms) {
        double t = a[npairs] * d[j];
        for (int c = 0; c < nchunk; ++c) t += tpart[int64_t(c) * n_atoms + j];
        Av[node[j]] -= kappa * t;
    }
}

// x = 0, r = rhs; partial rhs.rhs
__global__ void k_pcg_init(int64_t n, const double* rhs, double* x, double* r, double* part) {
    double bb = 0.0;
    NGRID_LOOP(i, n) {
        const double v = rhs[i];
        x[i] = 0.0;
        r[i] = v;
        bb += v * v;
    }
    const double t = block_sum(bb);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// z = M^-1 r with the Jacobi preconditioner
__global__ void k_jacobi(int64_t n, const double* minv, const double* r, double* z, const double* done) {
    if (done && *done != 0.0) return;
    NGRID_LOOP(i, n) z[i] = minv[i] * r[i];
}

// p = z; partial r.z
__global__ void k_pcg_first_p(int64_t n, const double* r, const double* z, double* p, double* part) {
    double rz = 0.0;
    NGRID_LOOP(i, n) {
        p[i] = z[i];
        rz += r[i] * z[i];
    }
    const double t = block_sum(rz);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void k_pcg_init_scalars(const double* part_bb, const double* part_rz, int64_t nb, double* s) {
    const double bb = sum_part(part_bb, nb);
    const double rz = sum_part(part_rz, nb);
    if (threadIdx.x != 0) return;
    for (int k = 0; k < NC_NS; ++k) s[k] = 0.0;
    s[NC_RZ] = rz;
    s[NC_BB] = bb;
    if (bb == 0.0) s[NC_DONE] = 1.0;   // G = 0: the step is zero
}

__global__ void k_pdot(int64_t n, const double* p, const double* Ap, double* part, const double* done) {
    if (*done != 0.0) return;
    double acc = 0.0;
    NGRID_LOOP(i, n) acc += p[i] * Ap[i];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void k_pcg_alpha(const double* part, int64_t nb, double* s) {
    if (s[NC_DONE] != 0.0) return;
    const double pap = sum_part(part, nb);
    if (threadIdx.x == 0) s[NC_ALPHA] = pap > 0.0 ? s[NC_RZ] / pap : 0.0;
}

// x += alpha p, r -= alpha Ap; partial r.r
__global__ void k_pcg_update(int64_t n, double* x, double* r, const double* p, const double* Ap, const double* s,
                             double* part) {
    if (s[NC_DONE] != 0.0) return;
    const double al = s[NC_ALPHA];
    double rr = 0.0;
    NGRID_LOOP(i, n) {
        x[i] += al * p[i];
        const double rv = r[i] - al * Ap[i];
        r[i] = rv;
        rr += rv * rv;
    }
    const double t = block_sum(rr);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// beta = r.z / previous r.z and the stopping test |r| <= rel_tol |rhs|
__global__ void k_pcg_beta(const double* part_rr, const double* part_rz, int64_t nb, double* s, double rel_tol,
                           int max_iter) {
    if (s[NC_DONE] != 0.0) return;
    const double rr = sum_part(part_rr, nb);
    const double rz = sum_part(part_rz, nb);
    if (threadIdx.x != 0) return;
    s[NC_BETA] = s[NC_RZ] != 0.0 ? rz / s[NC_RZ] : 0.0;
    s[NC_RZ] = rz;
    s[NC_ITERS] += 1.0;
    const double rel = s[NC_BB] > 0.0 ? sqrt(rr / s[NC_BB]) : 0.0;
    s[NC_REL] = rel;
    if (rel <= rel_tol || s[NC_ITERS] >= max_iter) s[NC_DONE] = 1.0;
}

__global__ void k_pcg_p(int64_t n, const double* z, double* p, const double* s) {
    if (s[NC_DONE] != 0.0) return;
    const double b = s[NC_BETA];
    NGRID_LOOP(i, n) p[i] = z[i] + b * p[i];
}

__global__ void k_scale_copy(int64_t n, double a, const double* x, double* y) {
    NGRID_LOOP(i, n) y[i] = a * x[i];
}

// partial dots of v with the m vectors base + l n: part[l * nb + block]
__global__ void k_multi_dot(int64_t n, const double* v, const double* base, double* part) {
    const int l = blockIdx.y;
    const double* w = base + int64_t(l) * n;
    double acc = 0.0;
    NGRID_LOOP(i, n) acc += v[i] * w[i];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[int64_t(l) * gridDim.x + blockIdx.x] = t;
}

__global__ void k_sum_rows(const double* part, int64_t nb, double* out) {
    const double t = sum_part(part + int64_t(blockIdx.x) * nb, nb);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// dX = U - X_prev, dF = f - F_prev into a history slot; X_prev = U, F_prev = f
__global__ void k_anderson_push(int64_t n, const double* U, const double* f, double* Xp, double* Fp, double* dX,
                                double* dF, int have_prev) {
    NGRID_LOOP(i, n) {
        if (have_prev) {
            dX[i] = U[i] - Xp[i];
            dF[i] = f[i] - Fp[i];
        }
        Xp[i] = U[i];
        Fp[i] = f[i];
    }
}

// U += f - sum_l gamma_l (dX_l + dF_l)
__global__ void k_anderson_update(int64_t n, double* U, const double* f, const double* dX, const double* dF,
                                  const double* gamma, int m) {
    NGRID_LOOP(i, n) {
        double u = U[i] + f[i];
        for (int l = 0; l < m; ++l) u -= gamma[l] * (dX[int64_t(l) * n + i] + dF[int64_t(l) * n + i]);
        U[i] = u;
    }
}

double fermi_occ(double E, double Ef, double kT) {
    const double t = (E - Ef) / kT;
    return t > 0 ? std::exp(-t) / (1.0 + std::exp(-t)) : 1.0 / (1.0 + std::exp(t));
}

double fermi_slope(double E, double Ef, double kT) {
    const double f = fermi_occ(E, Ef, kT);
    return -f * (1.0 - f) / kT;
}

// minimum-norm solution of the symmetric positive semi-definite system N g = r
// (m <= 8) by cyclic Jacobi eigen-decomposition; eigenvalues below 1e-12 of
// the largest are dropped (a least-squares solve of the Anderson problem)
std::vector<double> psd_solve(std::vector<double> N, const std::vector<double>& r, int m) {
    std::vector<double> V(static_cast<size_t>(m * m), 0.0);
    for (int i = 0; i < m; ++i) V[size_t(i * m + i)] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = i + 1; j < m; ++j) off += N[size_t(i * m + j)] * N[size_t(i * m + j)];
        if (off < 1e-300) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = N[size_t(p * m + q)];
                if (apq == 0.0) continue;
                const double th = 0.5 * (N[size_t(q * m + q)] - N[size_t(p * m + p)]) / apq;
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < m; ++k) {
                    const double akp = N[size_t(k * m + p)], akq = N[size_t(k * m + q)];
                    N[size_t(k * m + p)] = c * akp - s * akq;
                    N[size_t(k * m + q)] = s * akp + c * akq;
                }
                for (int k = 0; k < m; ++k) {
                    const double apk = N[size_t(p * m + k)], aqk = N[size_t(q * m + k)];
                    N[size_t(p * m + k)] = c * apk - s * aqk;
                    N[size_t(q * m + k)] = s * apk + c * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    const double vkp = V[size_t(k * m + p)], vkq = V[size_t(k * m + q)];
                    V[size_t(k * m + p)] = c * vkp - s * vkq;
                    V[size_t(k * m + q)] = s * vkp + c * vkq;
                }
            }
    }
    double lmax = 0.0;
    for (int i = 0; i < m; ++i) lmax = std::max(lmax, N[size_t(i * m + i)]);
    std::vector<double> g(static_cast<size_t>(m), 0.0);
    for (int e = 0; e < m; ++e) {
        const double lam = N[size_t(e * m + e)];
        if (!(lam > 1e-12 * lmax)) continue;
        double c = 0.0;
        for (int k = 0; k < m; ++k) c += V[size_t(k * m + e)] * r[size_t(k)];
        c /= lam;
        for (int k = 0; k < m; ++k) g[size_t(k)] += c * V[size_t(k * m + e)];
    }
    return g;
}

}  // namespace

void NewtonWork::reset() {
    have_prev = false;
    count = 0;
    head = 0;
}

void newton_update(hipStream_t st, NewtonWork& W, const NewtonIn& in, double* U, NewtonOut* out) {
    const int K = int(in.sel.size());
    const int64_t na = in.n_atoms;
    const int nx = in.grid[0], ny = in.grid[1], nz = in.grid[2];
    const int64_t n = int64_t(nx) * ny * nz;
    const int depth = in.depth;
    TBH_REQUIRE(depth >= 0 && depth <= 8, "Anderson depth must be 0..8");
    // --- coefficients of chi (host, K <= 128 states)
    std::vector<double> f(static_cast<size_t>(K)), fp(static_cast<size_t>(K));
    double fsum = 0.0;
    for (int i = 0; i < K; ++i) {
        f[size_t(i)] = fermi_occ(in.E[size_t(i)], in.Ef, in.kT);
        fp[size_t(i)] = fermi_slope(in.E[size_t(i)], in.Ef, in.kT);
        fsum += fp[size_t(i)];
    }
    std::vector<int2> pairs;
    std::vector<double> coef;
    std::vector<int> diag_pair(static_cast<size_t>(K));
    double cmax = 0.0;
    std::vector<double> call;
    for (int i = 0; i < K; ++i)
        for (int k = i; k < K; ++k) {
            const double dE = in.E[size_t(i)] - in.E[size_t(k)];
            double g;
            if (std::fabs(dE) <= 1e-5 * in.kT)
                g = fermi_slope(0.5 * (in.E[size_t(i)] + in.E[size_t(k)]), in.Ef, in.kT);
            else
                g = (f[size_t(i)] - f[size_t(k)]) / dE;
            const double c = (i == k ? 2.0 : 4.0) * g;
            call.push_back(c);
            cmax = std::max(cmax, std::fabs(c));
        }
    {
        size_t t = 0;
        for (int i = 0; i < K; ++i)
            for (int k = i; k < K; ++k, ++t) {
                const double c = call[t];
                if (i == k) {
                    diag_pair[size_t(i)] = int(pairs.size());
                } else if (!(std::fabs(c) > 1e-14 * cmax)) {
                    continue;
                }
                pairs.push_back(make_int2(i, k));
                coef.push_back(c);
            }
    }
    const int npairs = int(pairs.size());
    const double cd = (in.fixed || !(fsum < 0.0)) ? 0.0 : -2.0 / fsum;
    // --- device buffers
    W.R.alloc(size_t(std::max(npairs, 1)) * size_t(na) * 8);
    W.coef.alloc(size_t(npairs + 1) * 8);
    W.pairs.alloc(size_t(npairs + 1) * sizeof(int2));
    W.sel.alloc(size_t(K + 1) * 4);
    W.inv.alloc(size_t(K + 1) * 8);
    W.fp.alloc(size_t(K + 1) * 8);
    W.diag.alloc(size_t(K + 1) * 4);
    W.d.alloc(size_t(na) * 8);
    W.va.alloc(size_t(na) * 8);
    // sum_p a_p rho_p in chunks of pairs, enough workgroups to cover the chip
    const int nchunk = int(std::max<int64_t>(1, std::min<int64_t>(64, (2048 + blocks_for(na) - 1) / blocks_for(na))));
    const int per_chunk = (npairs + nchunk - 1) / nchunk;
    W.tpart.alloc(size_t(nchunk) * size_t(na) * 8);
    W.a.alloc(size_t(npairs + 1) * 8);
    W.minv.alloc(size_t(n) * 8);
    for (DevBuf* b : {&W.x, &W.r, &W.z, &W.p, &W.Ap, &W.G, &W.Xp, &W.Fp}) b->alloc(size_t(n) * 8);
    W.part.alloc(size_t(2 * 4096 + 2 * 8 * 4096) * 8);
    W.s.alloc(NC_NS * 8);
    W.small.alloc(32 * 8);
    if (depth > 0) {
        W.dX.alloc(size_t(depth) * size_t(n) * 8);
        W.dF.alloc(size_t(depth) * size_t(n) * 8);
    }
    if (K > 0) {
        TBH_HIP(hipMemcpyAsync(W.coef.p, coef.data(), size_t(npairs) * 8, hipMemcpyHostToDevice, st));
        TBH_HIP(hipMemcpyAsync(W.pairs.p, pairs.data(), size_t(npairs) * sizeof(int2), hipMemcpyHostToDevice, st));
        TBH_HIP(hipMemcpyAsync(W.sel.p, in.sel.data(), size_t(K) * 4, hipMemcpyHostToDevice, st));
        TBH_HIP(hipMemcpyAsync(W.inv.p, in.inv_norm.data(), size_t(K) * 8, hipMemcpyHostToDevice, st));
        TBH_HIP(hipMemcpyAsync(W.fp.p, fp.data(), size_t(K) * 8, hipMemcpyHostToDevice, st));
        TBH_HIP(hipMemcpyAsync(W.diag.p, diag_pair.data(), size_t(K) * 4, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_pair_density, dim3(unsigned(blocks_for(na)), unsigned(npairs)), dim3(TPB), 0, st,
                           in.Y, in.ns, in.n_o, na, W.pairs.as<int2>(), W.sel.as<int>(), W.inv.as<double>(),
                           W.R.as<double>());
    }
    const double inv_h2 = 1.0 / (in.h * in.h);
    const int64_t gn = blocks_for(n), ga = blocks_for(na);
    hipLaunchKernelGGL(k_fill, dim3(gn), dim3(TPB), 0, st, n, 1.0 / (6.0 * inv_h2), W.minv.as<double>());
    if (K > 0)
        hipLaunchKernelGGL(k_newton_diag, dim3(ga), dim3(TPB), 0, st, na, W.R.as<double>(), W.coef.as<double>(),
                           npairs, W.diag.as<int>(), W.fp.as<double>(), K, cd, in.kappa, 6.0 * inv_h2, in.node,
                           W.d.as<double>(), W.minv.as<double>());
    // --- G = A U + b (b = kappa (N_D - n)); J x = G by preconditioned CG from
    // x = 0; the Newton step is f = -x
    hipLaunchKernelGGL(k_apply_a, dim3(gn), dim3(TPB), 0, st, nx, ny, nz, inv_h2, U, in.b, W.G.as<double>(),
                       (const double*)nullptr);
    double* part = W.part.as<double>();
    double* s = W.s.as<double>();
    double* part2 = part + 4096;   // second set of partial sums (r.z)
    auto precondition = [&](const double* done) {
        if (in.pre)
            in.pre->solve(st, W.r.as<double>(), W.z.as<double>());
        else
            hipLaunchKernelGGL(k_jacobi, dim3(gn), dim3(TPB), 0, st, n, W.minv.as<double>(), W.r.as<double>(),
                               W.z.as<double>(), done);
    };
    hipLaunchKernelGGL(k_pcg_init, dim3(gn), dim3(TPB), 0, st, n, W.G.as<double>(), W.x.as<double>(),
                       W.r.as<double>(), part);
    precondition(nullptr);
    hipLaunchKernelGGL(k_pcg_first_p, dim3(gn), dim3(TPB), 0, st, n, W.r.as<double>(), W.z.as<double>(),
                       W.p.as<double>(), part2);
    hipLaunchKernelGGL(k_pcg_init_scalars, dim3(1), dim3(TPB), 0, st, part, part2, gn, s);
    double hs[NC_NS] = {};
    // the direct preconditioner leaves few iterations: check after each few
    const int chunk = in.pre ? 4 : 20;
    for (int it = 0; it < in.cg_max_iter; it += chunk) {
        for (int c = 0; c < chunk; ++c) {
            hipLaunchKernelGGL(k_apply_a, dim3(gn), dim3(TPB), 0, st, nx, ny, nz, inv_h2, W.p.as<double>(),
                               (const double*)nullptr, W.Ap.as<double>(), s + NC_DONE);
            if (K > 0) {
                hipLaunchKernelGGL(k_gather_nodes, dim3(ga), dim3(TPB), 0, st, na, in.node, W.p.as<double>(),
                                   W.va.as<double>(), s + NC_DONE);
                hipLaunchKernelGGL(k_pair_dot, dim3(unsigned(npairs + 1)), dim3(TPB), 0, st, na, W.R.as<double>(),
                                   npairs, W.va.as<double>(), W.d.as<double>(), W.coef.as<double>(), cd,
                                   W.a.as<double>(), s + NC_DONE);
                hipLaunchKernelGGL(k_chi_partial, dim3(unsigned(ga), unsigned(nchunk)), dim3(TPB), 0, st, na,
                                   W.R.as<double>(), npairs, per_chunk, W.a.as<double>(), W.tpart.as<double>(),
                                   s + NC_DONE);
                hipLaunchKernelGGL(k_chi_apply, dim3(ga), dim3(TPB), 0, st, na, nchunk, W.tpart.as<double>(), npairs,
                                   W.a.as<double>(), W.d.as<double>(), in.node, in.kappa, W.Ap.as<double>(),
                                   s + NC_DONE);
            }
            hipLaunchKernelGGL(k_pdot, dim3(gn), dim3(TPB), 0, st, n, W.p.as<double>(), W.Ap.as<double>(), part,
                               s + NC_DONE);
            hipLaunchKernelGGL(k_pcg_alpha, dim3(1), dim3(TPB), 0, st, part, gn, s);
            hipLaunchKernelGGL(k_pcg_update, dim3(gn), dim3(TPB), 0, st, n, W.x.as<double>(), W.r.as<double>(),
                               W.p.as<double>(), W.Ap.as<double>(), s, part);
            precondition(s + NC_DONE);
            hipLaunchKernelGGL(k_pdot, dim3(gn), dim3(TPB), 0, st, n, W.r.as<double>(), W.z.as<double>(), part2,
                               s + NC_DONE);
            hipLaunchKernelGGL(k_pcg_beta, dim3(1), dim3(TPB), 0, st, part, part2, gn, s, in.cg_tol, in.cg_max_iter);
            hipLaunchKernelGGL(k_pcg_p, dim3(gn), dim3(TPB), 0, st, n, W.z.as<double>(), W.p.as<double>(), s);
        }
        TBH_HIP(hipMemcpyAsync(hs, s, sizeof(hs), hipMemcpyDeviceToHost, st));
        TBH_HIP(hipStreamSynchronize(st));
        if (hs[NC_DONE] != 0.0) break;
    }
    double* fstep = W.z.as<double>();
    hipLaunchKernelGGL(k_scale_copy, dim3(gn), dim3(TPB), 0, st, n, -1.0, W.x.as<double>(), fstep);
    // --- Anderson mixing over the stored differences of iterates and steps
    double* gam = W.small.as<double>();
    if (depth == 0 || !W.have_prev) {
        if (depth > 0)
            hipLaunchKernelGGL(k_anderson_push, dim3(gn), dim3(TPB), 0, st, n, U, fstep, W.Xp.as<double>(),
                               W.Fp.as<double>(), (double*)nullptr, (double*)nullptr, 0);
        hipLaunchKernelGGL(k_anderson_update, dim3(gn), dim3(TPB), 0, st, n, U, fstep, (const double*)nullptr,
                           (const double*)nullptr, (const double*)nullptr, 0);
        W.have_prev = depth > 0;
    } else {
        const int slot = W.head;
        double* dX = W.dX.as<double>();
        double* dF = W.dF.as<double>();
        hipLaunchKernelGGL(k_anderson_push, dim3(gn), dim3(TPB), 0, st, n, U, fstep, W.Xp.as<double>(),
                           W.Fp.as<double>(), dX + int64_t(slot) * n, dF + int64_t(slot) * n, 1);
        W.head = (W.head + 1) % depth;
        W.count = std::min(W.count + 1, depth);
        // dF_new . dF_l and f . dF_l for every slot
        double* dots = W.small.as<double>() + 16;
        hipLaunchKernelGGL(k_multi_dot, dim3(unsigned(gn), unsigned(depth)), dim3(TPB), 0, st, n,
                           dF + int64_t(slot) * n, dF, part);
        hipLaunchKernelGGL(k_sum_rows, dim3(unsigned(depth)), dim3(TPB), 0, st, part, gn, dots);
        hipLaunchKernelGGL(k_multi_dot, dim3(unsigned(gn), unsigned(depth)), dim3(TPB), 0, st, n, fstep, dF,
                           part + int64_t(depth) * gn);
        hipLaunchKernelGGL(k_sum_rows, dim3(unsigned(depth)), dim3(TPB), 0, st, part + int64_t(depth) * gn, gn,
                           dots + 8);
        double hd[16];
        TBH_HIP(hipMemcpyAsync(hd, dots, 16 * 8, hipMemcpyDeviceToHost, st));
        TBH_HIP(hipStreamSynchronize(st));
        W.gram.resize(size_t(depth * depth));
        for (int l = 0; l < depth; ++l) {
            W.gram[size_t(slot * depth + l)] = hd[l];
            W.gram[size_t(l * depth + slot)] = hd[l];
        }
        // the valid slots: the count most recent ones
        const int m = W.count;
        std::vector<int> idx(static_cast<size_t>(m));
        for (int l = 0; l < m; ++l) idx[size_t(l)] = (slot - l + depth) % depth;
        std::vector<double> N(static_cast<size_t>(m * m)), r(static_cast<size_t>(m));
        for (int a = 0; a < m; ++a) {
            r[size_t(a)] = hd[8 + idx[size_t(a)]];
            for (int b2 = 0; b2 < m; ++b2) N[size_t(a * m + b2)] = W.gram[size_t(idx[size_t(a)] * depth + idx[size_t(b2)])];
        }
        const std::vector<double> g = psd_solve(N, r, m);
        std::vector<double> gfull(static_cast<size_t>(depth), 0.0);
        for (int a = 0; a < m; ++a) gfull[size_t(idx[size_t(a)])] = g[size_t(a)];
        TBH_HIP(hipMemcpyAsync(gam, gfull.data(), size_t(depth) * 8, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_anderson_update, dim3(gn), dim3(TPB), 0, st, n, U, fstep, dX, dF, gam, depth);
    }
    TBH_HIP(hipGetLastError());
    TBH_HIP(hipStreamSynchronize(st));
    if (out) {
        out->cg_iters = int(hs[NC_ITERS]);
        out->cg_rel = hs[NC_REL];
        out->npairs = npairs;
    }
}

}  // namespace tbh
