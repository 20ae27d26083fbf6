// Lanczos eigensolver for the states nearest a target energy, on the GPU.
//
// The paper's Schrodinger step finds eigenstates with an iterative Lanczos
// solver (Sec. III-A, item 1); its benchmarks time a fixed number of Lanczos
// iterations (Sec. II-B, Figs. 2-3).  Here every iteration runs on the device
// with no host round trip:
//
//   hx (fused):  w = H v_j - beta_j v_{j-1}, FP64 partials of Re(v_j^H w), |w|^2
//   scalars:     alpha_j; without reorthogonalisation beta_{j+1}^2 =
//                |w|^2 - alpha_j^2 (guarded: on cancellation the norm of
//                w - alpha_j v_j is taken explicitly, in the same kernel)
//   CGS2:        w -= alpha_j v_j, then twice { c = V^H w ; w -= V c } with
//                FP64 accumulation over FP32 (or FP64) stored vectors
//   next:        v_{j+1} = w / beta_{j+1}; breakdown if beta_{j+1} <= 1e-12 max|T|
//
// After the recurrence: FP64 Sturm bisection of the tridiagonal T (one
// thread per eigenvalue), candidates nearest sigma, FP64 inverse iteration
// for their eigenvectors, Ritz vectors y = V s in FP64, explicit residuals
// |H y - theta y| and Rayleigh quotients y^H H y with the FP64 copy of H.
// Every reduction is fixed-order (no atomics), so results are bitwise
// reproducible.
#include <chrono>
#include <cmath>

#include "tbh_internal.h"
#include "lanczos.h"

namespace tbh {

namespace {

constexpr int TPB = 256;

// sum NV doubles over a 256-thread block; result valid in thread 0
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*sh)[NV]) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = (sh[0][k] + sh[1][k]) + (sh[2][k] + sh[3][k]);
    __syncthreads();
}

// fixed-order sum of part[b * stride + off] over b < n by one block
__device__ double block_reduce_strided(const double* part, int64_t n, int stride, int off) {
    double v[1] = {0.0};
    for (int64_t b = threadIdx.x; b < n; b += TPB) v[0] += part[b * stride + off];
    __shared__ double sh[4][1];
    block_sum<1>(v, sh);
    return v[0];
}

// ---------------------------------------------------------------------------
// step scalars
// ---------------------------------------------------------------------------

// After the fused hx kernel: alpha_j and (without reorthogonalisation)
// beta_{j+1}.  The hx kernel leaves one (Re x^H y, |y|^2) pair per
// wavefront (16k pairs for a million atoms); one 1024-thread block sums both
// in a single pass of 16-byte loads with four independent accumulators per
// thread, in a fixed order.  beta_{j+1}^2 = |w|^2 - alpha_j^2 unless that
// cancels (below 1e-8 |w|^2); then the same block takes |w - alpha_j v_j|
// explicitly over the n scalars of w and v_j (slow, and only on that path).
constexpr int SCAL_TPB = 1024;

__device__ __forceinline__ double scal_block_sum(double v, double* sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < SCAL_TPB / 64; ++w) r += sh[w];
    return r;
}

template <typename T>
__global__ __launch_bounds__(SCAL_TPB) void k_step_scalars(const double* part, int64_t nblk, LzDev d, int j,
                                                           int reorth, const T* w, const T* vj, int64_t n) {
    if (d.ctrl[LZ_BREAK] != 0.0) return;
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2* p = reinterpret_cast<const d2*>(part);
    d2 s0 = {0.0, 0.0}, s1 = {0.0, 0.0}, s2 = {0.0, 0.0}, s3 = {0.0, 0.0};
    int64_t b = threadIdx.x;
    for (; b + 3 * SCAL_TPB < nblk; b += 4 * SCAL_TPB) {
        const d2 v0 = p[b], v1 = p[b + SCAL_TPB], v2 = p[b + 2 * SCAL_TPB], v3 = p[b + 3 * SCAL_TPB];
        s0 += v0;
        s1 += v1;
        s2 += v2;
        s3 += v3;
    }
    for (; b < nblk; b += SCAL_TPB) s0 += p[b];
    const d2 t = (s0 + s1) + (s2 + s3);
    __shared__ double sh[SCAL_TPB / 64];
    // every thread holds the block totals, so the branch below is uniform
    const double a = scal_block_sum(t.x, sh);
    const double ww = scal_block_sum(t.y, sh);
    const double tmax = fmax(d.ctrl[LZ_TMAX], fabs(a));
    if (reorth) {
        if (threadIdx.x == 0) {
            d.alpha[j] = a;
            d.ctrl[LZ_TMAX] = tmax;
        }
        return;
    }
    const double b2 = ww - a * a;
    double bb;
    if (b2 > 1e-8 * ww) {
        bb = sqrt(b2);
    } else {
        // cancellation: the norm of w - alpha_j v_j, explicitly
        double acc = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += SCAL_TPB) {
            const double u = double(w[i]) - a * double(vj[i]);
            acc += u * u;
        }
        bb = sqrt(scal_block_sum(acc, sh));
    }
    if (threadIdx.x != 0) return;
    d.alpha[j] = a;
    d.beta[j + 1] = bb;
    const double tm = fmax(tmax, bb);
    d.ctrl[LZ_TMAX] = tm;
    d.ctrl[LZ_STEPS] = j + 1;
    if (bb <= 1e-12 * tm) {
        d.ctrl[LZ_BREAK] = 1.0;
    } else {
        d.ctrl[LZ_INVB] = 1.0 / bb;
    }
}

// beta_{j+1} = sqrt(sum of explicit |w|^2 partials) (reorthogonalised path)
__global__ void k_finish_beta(const double* part, int64_t nblk, LzDev d, int j) {
    if (d.ctrl[LZ_BREAK] != 0.0) return;
    const double s = block_reduce_strided(part, nblk, 1, 0);
    if (threadIdx.x != 0) return;
    const double b = sqrt(s);
    d.beta[j + 1] = b;
    d.ctrl[LZ_TMAX] = fmax(d.ctrl[LZ_TMAX], b);
    d.ctrl[LZ_STEPS] = j + 1;
    if (b <= 1e-12 * d.ctrl[LZ_TMAX]) {
        d.ctrl[LZ_BREAK] = 1.0;
    } else {
        d.ctrl[LZ_INVB] = 1.0 / b;
    }
}

// ---------------------------------------------------------------------------
// vector kernels (n = number of real scalars; complex vectors interleaved)
// ---------------------------------------------------------------------------

// no reorthogonalisation: v_{j+1} = (w - alpha_j v_j) / beta_{j+1}
template <typename T>
__global__ void k_lz_next(int64_t n, const T* w, const T* vj, T* vn, LzDev d, int j) {
    if (d.ctrl[LZ_BREAK] != 0.0) return;
    const double a = d.alpha[j];
    const double ib = d.ctrl[LZ_INVB];
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB)
        vn[i] = T((double(w[i]) - a * double(vj[i])) * ib);
}

// v_{j+1} = w * (1/beta_{j+1}) (reorthogonalised path)
template <typename T>
__global__ void k_scale_next(int64_t n, const T* w, T* vn, LzDev d) {
    if (d.ctrl[LZ_BREAK] != 0.0) return;
    const double ib = d.ctrl[LZ_INVB];
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB)
        vn[i] = T(double(w[i]) * ib);
}

// w -= alpha_j v_j (before the first projection pass)
template <typename T>
__global__ void k_sub_alpha(int64_t n, T* w, const T* vj, LzDev d, int j) {
    if (d.ctrl[LZ_BREAK] != 0.0) return;
    const double a = d.alpha[j];
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB)
        w[i] = T(double(w[i]) - a * double(vj[i]));
}

// Classical Gram-Schmidt projections c_i = v_i^H w, i < nvec, as per-block
// partials part[(i * nrb + row_block) * CS + {re, im}].  The grid is
// (row blocks) x (groups of VG vectors); a block owns RPT * TPB consecutive
// elements and one group, so small dimensions with many vectors still fill
// the device.
template <typename T, bool CPLX, int VG, int RPT>
__global__ __launch_bounds__(TPB) void k_orth_dots(int64_t n_el, const T* V, int64_t ld, int nvec, const T* w,
                                                   LzDev d, double* part) {
    constexpr int CS = CPLX ? 2 : 1;
    if (d.ctrl[LZ_BREAK] != 0.0) return;
    const int64_t nrb = gridDim.x;
    const int64_t e0 = int64_t(blockIdx.x) * RPT * TPB + threadIdx.x;
    const int g0 = blockIdx.y * VG;
    double wr[RPT][CS];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int64_t e = e0 + int64_t(k) * TPB;
#pragma unroll
        for (int q = 0; q < CS; ++q) wr[k][q] = e < n_el ? double(w[e * CS + q]) : 0.0;
    }
    double acc[VG * CS];
#pragma unroll
    for (int t = 0; t < VG * CS; ++t) acc[t] = 0.0;
#pragma unroll
    for (int t = 0; t < VG; ++t) {
        const int i = g0 + t;
        if (i < nvec) {
            const T* vi = V + int64_t(i) * ld;
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const int64_t e = e0 + int64_t(k) * TPB;
                if (e < n_el) {
                    if constexpr (CPLX) {
                        const double vr = double(vi[2 * e]), vim = double(vi[2 * e + 1]);
                        acc[2 * t] += vr * wr[k][0] + vim * wr[k][1];
                        acc[2 * t + 1] += vr * wr[k][1] - vim * wr[k][0];
                    } else {
                        acc[t] += double(vi[e]) * wr[k][0];
                    }
                }
            }
        }
    }
    __shared__ double sh[4][VG * CS];
    block_sum<VG * CS>(acc, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int t = 0; t < VG; ++t)
            if (g0 + t < nvec)
#pragma unroll
                for (int q = 0; q < CS; ++q) part[((g0 + t) * nrb + blockIdx.x) * CS + q] = acc[t * CS + q];
    }
}

// c[i] = sum_b part[(i * nrb + b) * CS + q]: one block per coefficient
template <bool CPLX>
__global__ void k_orth_reduce(const double* part, int64_t nrb, double* c, const LzDev d) {
    constexpr int CS = CPLX ? 2 : 1;
    if (d.ctrl[LZ_BREAK] != 0.0) return;
    const int i = blockIdx.x;
    double v[CS];
#pragma unroll
    for (int q = 0; q < CS; ++q) v[q] = 0.0;
    for (int64_t b = threadIdx.x; b < nrb; b += TPB)
#pragma unroll
        for (int q = 0; q < CS; ++q) v[q] += part[(i * nrb + b) * CS + q];
    __shared__ double sh[4][CS];
    block_sum<CS>(v, sh);
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < CS; ++q) c[i * CS + q] = v[q];
}

// w -= V c over nvec vectors (FP64 accumulation); optional |w|^2 partials
template <typename T, bool CPLX>
__global__ __launch_bounds__(TPB) void k_orth_update(int64_t n_el, const T* V, int64_t ld, int nvec,
                                                     const double* c, T* w, LzDev d, double* part) {
    constexpr int CS = CPLX ? 2 : 1;
    if (d.ctrl[LZ_BREAK] != 0.0) return;
    extern __shared__ double cs_[];
    for (int t = threadIdx.x; t < nvec * CS; t += TPB) cs_[t] = c[t];
    __syncthreads();
    double nrm[1] = {0.0};
    for (int64_t e = blockIdx.x * int64_t(TPB) + threadIdx.x; e < n_el; e += int64_t(gridDim.x) * TPB) {
        double acc[CS];
#pragma unroll
        for (int q = 0; q < CS; ++q) acc[q] = double(w[e * CS + q]);
        for (int i = 0; i < nvec; ++i) {
            const T* vi = V + int64_t(i) * ld;
            if constexpr (CPLX) {
                const double vr = double(vi[2 * e]), vim = double(vi[2 * e + 1]);
                const double cr = cs_[2 * i], ci = cs_[2 * i + 1];
                acc[0] -= vr * cr - vim * ci;
                acc[1] -= vr * ci + vim * cr;
            } else {
                acc[0] -= double(vi[e]) * cs_[i];
            }
        }
#pragma unroll
        for (int q = 0; q < CS; ++q) {
            const T u = T(acc[q]);
            w[e * CS + q] = u;
            nrm[0] += double(u) * double(u);
        }
    }
    if (part) {
        __shared__ double sh[4][1];
        block_sum<1>(nrm, sh);
        if (threadIdx.x == 0) part[blockIdx.x] = nrm[0];
    }
}

// start vector: part = |v0|^2 partials (v0 in FP64)
__global__ void k_norm2(int64_t n, const double* v, double* part) {
    double acc[1] = {0.0};
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB)
        acc[0] += v[i] * v[i];
    __shared__ double sh[4][1];
    block_sum<1>(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

template <typename T>
__global__ void k_start(int64_t n, const double* v0, const double* part, int64_t nblk, T* out) {
    __shared__ double inv;
    const double s = block_reduce_strided(part, nblk, 1, 0);
    if (threadIdx.x == 0) inv = 1.0 / sqrt(s);
    __syncthreads();
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB)
        out[i] = T(v0[i] * inv);
}

template <typename T>
__global__ void k_cast_to_f64(int64_t n, const T* a, double* b) {
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB)
        b[i] = double(a[i]);
}

// ---------------------------------------------------------------------------
// FP64 tridiagonal eigensolver
// ---------------------------------------------------------------------------

// number of eigenvalues of T below x (Sturm count of the LDL^T pivots)
__device__ int sturm_count(int m, const double* a, const double* b, double x, double pivmin) {
    int cnt = 0;
    double q = a[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
    for (int i = 1; i < m; ++i) {
        q = a[i] - x - (b[i] * b[i]) / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0) ++cnt;
    }
    return cnt;
}

// beta[i] couples rows i-1 and i (beta[0] unused)
__global__ void k_bisect(int m, const double* alpha, const double* beta, double* theta) {
    const int k = blockIdx.x * TPB + threadIdx.x;
    if (k >= m) return;
    double lo = INFINITY, hi = -INFINITY, tn = 0.0;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? fabs(beta[i]) : 0.0) + (i + 1 < m ? fabs(beta[i + 1]) : 0.0);
        lo = fmin(lo, alpha[i] - r);
        hi = fmax(hi, alpha[i] + r);
        tn = fmax(tn, fabs(alpha[i]) + r);
    }
    const double eps = 2.220446049250313e-16;
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, tn * tn);
    lo -= 2 * eps * tn + 1e-300;
    hi += 2 * eps * tn + 1e-300;
    // find the (k+1)-th smallest: smallest x with count(x) >= k+1
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (hi - lo <= 2 * eps * fmax(fabs(lo), fabs(hi))) break;
        if (sturm_count(m, alpha, beta, mid, pivmin) >= k + 1)
            hi = mid;
        else
            lo = mid;
    }
    theta[k] = 0.5 * (lo + hi);
}

// the ncand eigenvalues nearest sigma (ties: smaller index), one thread
__global__ void k_select(int m, const double* theta, double sigma, int ncand, int* idx) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int hi = 0;
    while (hi < m && theta[hi] < sigma) ++hi;
    int lo = hi - 1;
    for (int c = 0; c < ncand; ++c) {
        const bool take_lo = lo >= 0 && (hi >= m || fabs(theta[lo] - sigma) <= fabs(theta[hi] - sigma));
        idx[c] = take_lo ? lo-- : hi++;
    }
}

// inverse iteration (T - theta I) s = b with partial-pivot LU; one thread per
// candidate; work: [ncand][5m] scratch
__global__ void k_invit(int m, const double* alpha, const double* beta, const double* theta,
                        const int* idx, int ncand, double* S, double* work) {
    const int c = blockIdx.x * TPB + threadIdx.x;
    if (c >= ncand) return;
    const double th = theta[idx[c]];
    double tn = 0.0;
    for (int i = 0; i < m; ++i)
        tn = fmax(tn, fabs(alpha[i]) + (i > 0 ? fabs(beta[i]) : 0.0) + (i + 1 < m ? fabs(beta[i + 1]) : 0.0));
    const double tiny = fmax(tn, 1e-300) * 2.220446049250313e-16;
    double* d = work + int64_t(c) * 5 * m;  // diagonal of U
    double* u1 = d + m;                      // first superdiagonal
    double* u2 = u1 + m;                     // second superdiagonal (from pivoting)
    double* l = u2 + m;                      // multipliers
    double* piv = l + m;                     // 1 if rows i, i+1 swapped
    // LU of T - th I (LAPACK dlagtf-style elimination)
    double dcur = alpha[0] - th, ucur = m > 1 ? beta[1] : 0.0;
    for (int i = 0; i < m - 1; ++i) {
        const double sub = beta[i + 1];
        const double dnext = alpha[i + 1] - th;
        const double unext = i + 2 < m ? beta[i + 2] : 0.0;
        if (fabs(dcur) >= fabs(sub)) {
            const double p = fabs(dcur) < tiny ? tiny : dcur;
            l[i] = sub / p;
            d[i] = p;
            u1[i] = ucur;
            u2[i] = 0.0;
            piv[i] = 0.0;
            dcur = dnext - l[i] * ucur;
            ucur = unext;
        } else {
            l[i] = dcur / sub;
            d[i] = sub;
            u1[i] = dnext;
            u2[i] = unext;
            piv[i] = 1.0;
            dcur = ucur - l[i] * dnext;
            ucur = -l[i] * unext;
        }
    }
    d[m - 1] = fabs(dcur) < tiny ? tiny : dcur;
    double* s = S + int64_t(c) * m;
    for (int i = 0; i < m; ++i) s[i] = 1.0 / sqrt(double(m)) * (1.0 + 0.01 * double(i % 7));
    for (int it = 0; it < 3; ++it) {
        // forward: apply L^{-1} with the recorded row swaps
        for (int i = 0; i < m - 1; ++i) {
            if (piv[i] != 0.0) {
                const double t = s[i];
                s[i] = s[i + 1];
                s[i + 1] = t - l[i] * s[i];
            } else {
                s[i + 1] -= l[i] * s[i];
            }
        }
        // back substitution with U (diag d, super u1, u2)
        s[m - 1] /= d[m - 1];
        if (m > 1) s[m - 2] = (s[m - 2] - u1[m - 2] * s[m - 1]) / d[m - 2];
        for (int i = m - 3; i >= 0; --i) s[i] = (s[i] - u1[i] * s[i + 1] - u2[i] * s[i + 2]) / d[i];
        double nr = 0.0;
        for (int i = 0; i < m; ++i) nr += s[i] * s[i];
        nr = 1.0 / sqrt(nr);
        for (int i = 0; i < m; ++i) s[i] *= nr;
    }
}

// Ritz vectors Y[c] = sum_i S[c][i] V[i] (FP64), candidates in groups of CG
template <typename T, int CG>
__global__ __launch_bounds__(TPB) void k_ritz(int64_t n, const T* V, int64_t ld, int m, const double* S,
                                              int ncand, double* Y) {
    const int c0 = blockIdx.y * CG;
    for (int64_t e = blockIdx.x * int64_t(TPB) + threadIdx.x; e < n; e += int64_t(gridDim.x) * TPB) {
        double acc[CG];
#pragma unroll
        for (int t = 0; t < CG; ++t) acc[t] = 0.0;
        for (int i = 0; i < m; ++i) {
            const double v = double(V[int64_t(i) * ld + e]);
#pragma unroll
            for (int t = 0; t < CG; ++t)
                if (c0 + t < ncand) acc[t] += S[int64_t(c0 + t) * m + i] * v;
        }
#pragma unroll
        for (int t = 0; t < CG; ++t)
            if (c0 + t < ncand) Y[int64_t(c0 + t) * n + e] = acc[t];
    }
}

// partials of |y|^2, Re(y^H z), |z - theta y|^2 for candidate c
__global__ void k_resid(int64_t n, const double* y, const double* z, const double* theta, const int* idx,
                        int c, double* part) {
    const double th = theta[idx[c]];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB) {
        const double a = y[i], b = z[i];
        acc[0] += a * a;
        acc[1] += a * b;
        const double r = b - th * a;
        acc[2] += r * r;
    }
    __shared__ double sh[4][3];
    block_sum<3>(acc, sh);
    if (threadIdx.x == 0)
        for (int q = 0; q < 3; ++q) part[blockIdx.x * 3 + q] = acc[q];
}

__global__ void k_resid_reduce(const double* part, int64_t nblk, const double* theta, const int* idx,
                               int c, double* out /* [ncand][4]: theta, res, refined, |y| */) {
    const double yy = block_reduce_strided(part, nblk, 3, 0);
    const double yz = block_reduce_strided(part, nblk, 3, 1);
    const double rr = block_reduce_strided(part, nblk, 3, 2);
    if (threadIdx.x == 0) {
        out[c * 4 + 0] = theta[idx[c]];
        out[c * 4 + 1] = sqrt(rr / yy);
        out[c * 4 + 2] = yz / yy;
        out[c * 4 + 3] = sqrt(yy);
    }
}

__global__ void k_scale_copy(int64_t n, const double* a, double s, double* b) {
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB)
        b[i] = a[i] * s;
}

int64_t grid_for(int64_t n) {
    int64_t g = (n + TPB - 1) / TPB;
    return g < 1 ? 1 : (g > 8192 ? 8192 : g);
}

}  // namespace

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------


void LzWork::ensure(const Ham& h, int steps, bool with_reorth, bool keep_basis) {
    const bool want_full = with_reorth || keep_basis;
    if (m == steps && reorth == with_reorth && full == want_full && V.p && dim == h.dim) return;
    drop_graph();
    dim = h.dim;
    const int64_t ns = h.dim * (h.cplx_h ? 2 : 1);
    const size_t esz = h.prec == TBH_F64 ? 8 : 4;
    TBH_REQUIRE(!with_reorth || steps <= 4000, "full reorthogonalisation supports at most 4000 steps");
    const int64_t nvec = want_full ? int64_t(steps) + 1 : 3;
    V.alloc(size_t(nvec) * ns * esz);
    w.alloc(size_t(ns) * esz);
    scal.alloc(sizeof(double) * (2 * size_t(steps) + 2 + LZ_NCTRL));
    const int64_t nblk_hx = hx_num_blocks(h.lay);
    const int64_t n_el = h.dim;
    const int64_t nrb = (n_el + 4 * TPB - 1) / (4 * TPB);
    size_t part_n = std::max<size_t>(2 * nblk_hx, 8192 * 3);
    if (with_reorth) part_n = std::max<size_t>(part_n, size_t(steps + 1) * nrb * 2);
    part.alloc(part_n * sizeof(double));
    coef.alloc(sizeof(double) * 2 * (size_t(steps) + 1));
    m = steps;
    reorth = with_reorth;
    full = want_full;
}

LzDev LzWork::dev(int m_) const {
    LzDev d;
    double* s = scal.as<double>();
    d.alpha = s;
    d.beta = s + m_;
    d.ctrl = s + 2 * m_ + 2;
    return d;
}

namespace {

__global__ void k_zero(int64_t n, double* a) {
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB) a[i] = 0.0;
}

// Every launch of an m-step recurrence, enqueued on st.  With ev non-null
// the H.x launches are bracketed by events (direct launches only).
void enqueue_recurrence(Ham& h, LzWork& W, int m, bool reorth, const double* v0_dev, hipStream_t st,
                        std::vector<hipEvent_t>* ev) {
    const bool f64 = h.prec == TBH_F64;
    const bool cx = h.cplx_h;
    const int cs = cx ? 2 : 1;
    const int64_t n_el = h.dim, ns = n_el * cs;
    const size_t esz = f64 ? 8 : 4;
    LzDev d = W.dev(m);
    const int64_t nscal = int64_t(W.scal.bytes / sizeof(double));
    hipLaunchKernelGGL(k_zero, dim3(grid_for(nscal)), dim3(TPB), 0, st, nscal, W.scal.as<double>());
    double* part = W.part.as<double>();
    // v_0 = v0 / |v0|
    char* Vb = W.V.as<char>();
    auto vec = [&](int64_t i) -> void* { return Vb + size_t(i) * ns * esz; };
    {
        const int64_t g = grid_for(ns);
        hipLaunchKernelGGL(k_norm2, dim3(g), dim3(TPB), 0, st, ns, v0_dev, part);
        if (f64)
            hipLaunchKernelGGL(k_start<double>, dim3(g), dim3(TPB), 0, st, ns, v0_dev, part, g,
                               static_cast<double*>(vec(0)));
        else
            hipLaunchKernelGGL(k_start<float>, dim3(g), dim3(TPB), 0, st, ns, v0_dev, part, g,
                               static_cast<float*>(vec(0)));
    }
    const int64_t nblk_hx = hx_num_blocks(h.lay);
    const int64_t gv = grid_for(ns);
    // the whole basis, or three rotating vectors
    const bool full = W.full;
    int iprev = 2, icur = 0, inext = 1;
    for (int j = 0; j < m; ++j) {
        void* vj = full ? vec(j) : vec(icur);
        void* vp = j == 0 ? nullptr : (full ? vec(j - 1) : vec(iprev));
        void* vn = full ? vec(j + 1) : vec(inext);
        HxArgs a;
        a.blocks = h.blocks.p;
        a.nbr = h.nbr_d.as<int32_t>();
        a.keys = h.keys_d.as<uint8_t>();
        a.x = vj;
        a.y = W.w.p;
        a.pot = h.has_pot ? h.pot_d.as<double>() : nullptr;
        a.n_atoms = h.n;
        a.xprev = vp;
        a.beta = d.beta + j;
        a.partial = part;
        if (ev) TBH_HIP(hipEventRecord((*ev)[2 * j], st));
        hx_launch(h.lay, f64, a, st);
        if (ev) TBH_HIP(hipEventRecord((*ev)[2 * j + 1], st));
        if (f64)
            hipLaunchKernelGGL(k_step_scalars<double>, dim3(1), dim3(SCAL_TPB), 0, st, part, nblk_hx, d, j,
                               int(reorth), W.w.as<double>(), static_cast<const double*>(vj), ns);
        else
            hipLaunchKernelGGL(k_step_scalars<float>, dim3(1), dim3(SCAL_TPB), 0, st, part, nblk_hx, d, j,
                               int(reorth), W.w.as<float>(), static_cast<const float*>(vj), ns);
        if (!reorth) {
            if (f64)
                hipLaunchKernelGGL(k_lz_next<double>, dim3(gv), dim3(TPB), 0, st, ns, W.w.as<double>(),
                                   static_cast<const double*>(vj), static_cast<double*>(vn), d, j);
            else
                hipLaunchKernelGGL(k_lz_next<float>, dim3(gv), dim3(TPB), 0, st, ns, W.w.as<float>(),
                                   static_cast<const float*>(vj), static_cast<float*>(vn), d, j);
            const int t = iprev;
            iprev = icur;
            icur = inext;
            inext = t;
        } else {
            orth_cgs2(h, W, d, j, st);
            if (f64)
                hipLaunchKernelGGL(k_scale_next<double>, dim3(gv), dim3(TPB), 0, st, ns,
                                   W.w.as<double>(), static_cast<double*>(vn), d);
            else
                hipLaunchKernelGGL(k_scale_next<float>, dim3(gv), dim3(TPB), 0, st, ns,
                                   W.w.as<float>(), static_cast<float*>(vn), d);
        }
    }
    TBH_HIP(hipGetLastError());
}

}  // namespace

void LzWork::drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
}

LzWork::~LzWork() {
    drop_graph();
    if (cap) (void)hipStreamDestroy(cap);
}

void lanczos_recurrence(Ham& h, LzWork& W, int m, bool reorth, const double* v0_dev,
                        double* alpha_h, double* beta_h, int* steps_h, int* breakdown_h, double* hx_ms,
                        bool keep_basis) {
    hipStream_t st = h.ctx->stream;
    W.ensure(h, m, reorth, keep_basis);
    if (hx_ms) {
        // timed: direct launches with events around every H.x
        std::vector<hipEvent_t> ev(2 * size_t(m));
        for (auto& e : ev) TBH_HIP(hipEventCreate(&e));
        enqueue_recurrence(h, W, m, reorth, v0_dev, st, &ev);
        TBH_HIP(hipStreamSynchronize(st));
        *hx_ms = 0.0;
        for (int j = 0; j < m; ++j) {
            float ms = 0.f;
            TBH_HIP(hipEventElapsedTime(&ms, ev[2 * j], ev[2 * j + 1]));
            *hx_ms += ms;
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
    } else {
        // the launch sequence depends only on these pointers and sizes: capture
        // it once into a graph and replay it on later calls
        const std::vector<const void*> key = {h.blocks.p, h.nbr_d.p, h.has_pot ? h.pot_d.p : nullptr, v0_dev,
                                              W.V.p, W.w.p, W.scal.p, W.part.p, W.coef.p,
                                              reinterpret_cast<const void*>(intptr_t(m)),
                                              reinterpret_cast<const void*>(intptr_t(reorth)),
                                              reinterpret_cast<const void*>(intptr_t(W.full))};
        if (!W.exec || key != W.key) {
            W.drop_graph();
            if (!W.cap) TBH_HIP(hipStreamCreateWithFlags(&W.cap, hipStreamNonBlocking));
            TBH_HIP(hipStreamBeginCapture(W.cap, hipStreamCaptureModeThreadLocal));
            try {
                enqueue_recurrence(h, W, m, reorth, v0_dev, W.cap, nullptr);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(W.cap, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            TBH_HIP(hipStreamEndCapture(W.cap, &W.graph));
            TBH_HIP(hipGraphInstantiate(&W.exec, W.graph, nullptr, nullptr, 0));
            W.key = key;
        }
        TBH_HIP(hipGraphLaunch(W.exec, st));
    }
    std::vector<double> s(W.scal.bytes / sizeof(double));
    TBH_HIP(hipMemcpyAsync(s.data(), W.scal.p, W.scal.bytes, hipMemcpyDeviceToHost, st));
    TBH_HIP(hipStreamSynchronize(st));
    const int steps = int(s[2 * m + 2 + LZ_STEPS]);
    if (steps_h) *steps_h = steps;
    if (breakdown_h) *breakdown_h = s[2 * m + 2 + LZ_BREAK] != 0.0;
    if (alpha_h)
        for (int j = 0; j < m; ++j) alpha_h[j] = j < steps ? s[j] : 0.0;
    if (beta_h)
        for (int j = 0; j < m; ++j) beta_h[j] = j < steps ? s[m + j + 1] : 0.0;
}

void orth_cgs2(Ham& h, LzWork& W, const LzDev& d, int j, hipStream_t st) {
    const bool f64 = h.prec == TBH_F64;
    const bool cx = h.cplx_h;
    const int64_t n_el = h.dim;
    const int64_t ld = n_el * (cx ? 2 : 1);
    constexpr int RPT = 4, VG = 8;
    const int64_t nrb = (n_el + RPT * TPB - 1) / (RPT * TPB);
    const int nvec = j + 1;
    const dim3 gd(unsigned(nrb), unsigned((nvec + VG - 1) / VG));
    double* part = W.part.as<double>();
    double* c = W.coef.as<double>();
    const int64_t gu = grid_for(n_el);
    const int64_t gv = grid_for(ld);
    const size_t shm = sizeof(double) * (cx ? 2 : 1) * size_t(nvec);
    if (f64)
        hipLaunchKernelGGL(k_sub_alpha<double>, dim3(gv), dim3(TPB), 0, st, ld, W.w.as<double>(),
                           W.V.as<double>() + int64_t(j) * ld, d, j);
    else
        hipLaunchKernelGGL(k_sub_alpha<float>, dim3(gv), dim3(TPB), 0, st, ld, W.w.as<float>(),
                           W.V.as<float>() + int64_t(j) * ld, d, j);
    for (int pass = 0; pass < 2; ++pass) {
#define TBH_ORTH(T, CX)                                                                               \
    hipLaunchKernelGGL((k_orth_dots<T, CX, VG, RPT>), gd, dim3(TPB), 0, st, n_el,                     \
                       static_cast<const T*>(W.V.p), ld, nvec, W.w.as<T>(), d, part);                 \
    hipLaunchKernelGGL((k_orth_reduce<CX>), dim3(nvec), dim3(TPB), 0, st, part, nrb, c, d);          \
    hipLaunchKernelGGL((k_orth_update<T, CX>), dim3(gu), dim3(TPB), shm, st, n_el,                    \
                       static_cast<const T*>(W.V.p), ld, nvec, c, W.w.as<T>(), d,                     \
                       pass == 1 ? part : nullptr);
        if (f64) {
            if (cx) { TBH_ORTH(double, true) } else { TBH_ORTH(double, false) }
        } else {
            if (cx) { TBH_ORTH(float, true) } else { TBH_ORTH(float, false) }
        }
#undef TBH_ORTH
    }
    hipLaunchKernelGGL(k_finish_beta, dim3(1), dim3(TPB), 0, st, part, gu, d, j);
}

void tridiag_gpu(hipStream_t st, int m, const double* alpha_d, const double* beta_d, double* theta_d) {
    hipLaunchKernelGGL(k_bisect, dim3((m + TPB - 1) / TPB), dim3(TPB), 0, st, m, alpha_d, beta_d, theta_d);
    TBH_HIP(hipGetLastError());
}

void ritz_pairs(Ham& h, LzWork& W, int steps, double sigma, int ncand, RitzOut& out) {
    TBH_REQUIRE(W.full && steps <= W.m, "Ritz vectors need the whole Lanczos basis");
    hipStream_t st = h.ctx->stream;
    const bool f64 = h.prec == TBH_F64;
    const bool cx = h.cplx_h;
    const int64_t ns = h.dim * (cx ? 2 : 1);
    const int m = W.m;
    LzDev d = W.dev(m);
    out.theta_all.alloc(sizeof(double) * steps);
    out.idx.alloc(sizeof(int) * ncand);
    out.S.alloc(sizeof(double) * size_t(ncand) * steps);
    out.work.alloc(sizeof(double) * size_t(ncand) * 5 * steps);
    out.Y.alloc(sizeof(double) * size_t(ncand) * ns);
    out.Z.alloc(sizeof(double) * size_t(ns));
    out.res.alloc(sizeof(double) * 4 * size_t(ncand));
    double* th = out.theta_all.as<double>();
    tridiag_gpu(st, steps, d.alpha, d.beta, th);
    hipLaunchKernelGGL(k_select, dim3(1), dim3(64), 0, st, steps, th, sigma, ncand, out.idx.as<int>());
    hipLaunchKernelGGL(k_invit, dim3((ncand + TPB - 1) / TPB), dim3(TPB), 0, st, steps, d.alpha, d.beta, th,
                       out.idx.as<int>(), ncand, out.S.as<double>(), out.work.as<double>());
    constexpr int CG = 8;
    const int64_t g = grid_for(ns);
    dim3 grid(g, (ncand + CG - 1) / CG);
    if (f64)
        hipLaunchKernelGGL((k_ritz<double, CG>), grid, dim3(TPB), 0, st, ns, W.V.as<double>(), ns, steps,
                           out.S.as<double>(), ncand, out.Y.as<double>());
    else
        hipLaunchKernelGGL((k_ritz<float, CG>), grid, dim3(TPB), 0, st, ns, W.V.as<float>(), ns, steps,
                           out.S.as<double>(), ncand, out.Y.as<double>());
    TBH_HIP(hipGetLastError());
    double* part = W.part.as<double>();
    for (int c = 0; c < ncand; ++c) {
        double* y = out.Y.as<double>() + size_t(c) * ns;
        HxArgs a;
        a.blocks = f64 ? h.blocks.p : h.blocks64.p;
        a.keys = h.keys_d.as<uint8_t>();
        a.nbr = h.nbr_d.as<int32_t>();
        a.x = y;
        a.y = out.Z.p;
        a.pot = h.has_pot ? h.pot_d.as<double>() : nullptr;
        a.n_atoms = h.n;
        hx_launch(f64 ? h.lay : h.lay64, true, a, st);
        hipLaunchKernelGGL(k_resid, dim3(g), dim3(TPB), 0, st, ns, y, out.Z.as<double>(), th,
                           out.idx.as<int>(), c, part);
        hipLaunchKernelGGL(k_resid_reduce, dim3(1), dim3(TPB), 0, st, part, g, th, out.idx.as<int>(), c,
                           out.res.as<double>());
    }
    TBH_HIP(hipGetLastError());
}

void scale_copy(hipStream_t st, int64_t n, const double* src, double s, double* dst) {
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(TPB), 0, st, n, src, s, dst);
    TBH_HIP(hipGetLastError());
}

void cast_to_f64(hipStream_t st, bool f64, int64_t n, const void* a, double* b) {
    const int64_t g = grid_for(n);
    if (f64)
        hipLaunchKernelGGL(k_cast_to_f64<double>, dim3(g), dim3(TPB), 0, st, n, static_cast<const double*>(a), b);
    else
        hipLaunchKernelGGL(k_cast_to_f64<float>, dim3(g), dim3(TPB), 0, st, n, static_cast<const float*>(a), b);
}

}  // namespace tbh
