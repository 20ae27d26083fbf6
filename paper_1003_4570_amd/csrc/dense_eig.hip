// Dense FP64 symmetric eigensolver for the projected matrix of block Lanczos
// (the Rayleigh-Ritz step of the block form of Sec. III-A item 1's Lanczos
// solver): the eigenpairs of an n x n real symmetric matrix nearest a target.
//
//  1. Householder reduction to tridiagonal form, T = Q^T A Q with
//     Q = H_0 H_1 ... H_{n-2}, H_k = I - tau_k v_k v_k^T (one workgroup; the
//     matrix, at most 2048^2 doubles, stays in L2);
//  2. the eigenvalues of the tridiagonal nearest the target by Sturm-count
//     multisection (one wavefront per eigenvalue, a window of 2 nc around
//     the target's index);
//  3. their eigenvectors by inverse iteration with partial-pivot LU, from
//     SplitMix64 start vectors that differ per candidate; candidates whose
//     eigenvalues lie within 1e-8 |T| of each other (numerically degenerate,
//     where inverse iteration alone cannot tell the vectors apart) are
//     orthogonalised among themselves;
//  4. back-transformation z = Q s.
// Every step is FP64 with fixed-order reductions (bitwise reproducible).
#include "dense_eig.h"

namespace tbh {

namespace {

constexpr int HT = 1024;      // threads of the Householder workgroup
constexpr int MAXN = 2048;    // largest matrix

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// sum over the workgroup (blockDim.x a multiple of 64, at most 1024); every
// thread receives the result
__device__ double wg_sum(double v, double* sh) {
    v = wave_sum(v);
    const int nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += sh[w];
        sh[16] = s;
    }
    __syncthreads();
    const double r = sh[16];
    __syncthreads();
    return r;
}

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Householder tridiagonalisation of the symmetric A (row-major, both
// triangles, overwritten).  d[n], e[n-1] (e[k] couples k and k+1), tau[n-1],
// V[k][0..n-k-2] = v_k (v_k[0] = 1) acting on rows k+1..n-1.
__global__ __launch_bounds__(HT) void k_sytrd(int n, double* __restrict__ A, double* __restrict__ d,
                                              double* __restrict__ e, double* __restrict__ tau,
                                              double* __restrict__ V) {
    __shared__ double v[MAXN], w[MAXN], sh[17];
    const int t = threadIdx.x;
    for (int k = 0; k + 1 < n; ++k) {
        const int m = n - k - 1;
        const double* xrow = A + int64_t(k) * n + k + 1;   // row k right of the diagonal = column k below it
        double ss = 0.0;
        for (int i = 1 + t; i < m; i += HT) ss += xrow[i] * xrow[i];
        ss = wg_sum(ss, sh);
        const double alpha = xrow[0];
        double tk = 0.0, beta = alpha, scal = 0.0;
        if (ss > 0.0) {
            const double nrm = sqrt(alpha * alpha + ss);
            beta = alpha >= 0.0 ? -nrm : nrm;
            tk = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        for (int i = t; i < m; i += HT) {
            const double vi = i == 0 ? 1.0 : (ss > 0.0 ? xrow[i] * scal : 0.0);
            v[i] = vi;
            V[int64_t(k) * n + i] = vi;
        }
        if (t == 0) {
            d[k] = A[int64_t(k) * n + k];
            e[k] = beta;
            tau[k] = tk;
        }
        __syncthreads();
        if (tk != 0.0) {
            // p = tau A22 v; A22 is symmetric, so p_i = tau sum_j A22[j][i] v_j
            double* A22 = A + int64_t(k + 1) * n + k + 1;
            double pv = 0.0;
            for (int i = t; i < m; i += HT) {
                double acc = 0.0;
                for (int j = 0; j < m; ++j) acc += A22[int64_t(j) * n + i] * v[j];
                w[i] = tk * acc;
                pv += w[i] * v[i];
            }
            pv = wg_sum(pv, sh);
            const double K = 0.5 * tk * pv;
            for (int i = t; i < m; i += HT) w[i] -= K * v[i];
            __syncthreads();
            // A22 -= v w^T + w v^T
            for (int i = t; i < m; i += HT) {
                const double vi = v[i], wi = w[i];
                for (int j = 0; j < m; ++j) A22[int64_t(j) * n + i] -= v[j] * wi + w[j] * vi;
            }
        }
        __syncthreads();
    }
    if (t == 0) d[n - 1] = A[int64_t(n - 1) * n + n - 1];
}

// The same reduction for n <= 64 (the Rayleigh-Ritz matrices of the filtered
// solver) on one wavefront with the matrix in LDS: lane c owns column c.  The
// products and updates run over all 64 rows with v and w zero outside the
// active block, so their loops have fixed bounds and every LDS access of a
// step is independent of the others; the sums over rows are in ascending row
// order as in k_sytrd, the two scalar sums are wavefront reductions.
constexpr int SMALLN = 64;

__global__ __launch_bounds__(64) void k_sytrd_lds(int n, double* __restrict__ A, double* __restrict__ d,
                                                  double* __restrict__ e, double* __restrict__ tau,
                                                  double* __restrict__ V) {
    __shared__ double As[SMALLN][SMALLN + 1];
    __shared__ double va[SMALLN], wa[SMALLN];
    const int c = threadIdx.x;
    const bool cin = c < n;
    for (int j = 0; j < SMALLN; ++j) As[j][c] = (j < n && cin) ? A[j * n + c] : 0.0;
    __syncthreads();
    for (int k = 0; k + 1 < n; ++k) {
        const bool act = c > k && cin;              // column k + 1 + i of the trailing block
        const double xc = act ? As[k][c] : 0.0;     // x_i, row k right of the diagonal
        const double ss = wave_sum(c > k + 1 && cin ? xc * xc : 0.0);
        const double alpha = As[k][k + 1];
        double tk = 0.0, beta = alpha, scal = 0.0;
        if (ss > 0.0) {
            const double nrm = sqrt(alpha * alpha + ss);
            beta = alpha >= 0.0 ? -nrm : nrm;
            tk = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
        }
        const double vc = act ? (c == k + 1 ? 1.0 : (ss > 0.0 ? xc * scal : 0.0)) : 0.0;
        if (act) V[int64_t(k) * n + (c - k - 1)] = vc;
        if (c == 0) {
            d[k] = As[k][k];
            e[k] = beta;
            tau[k] = tk;
        }
        va[c] = vc;
        __syncthreads();
        if (tk != 0.0) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < SMALLN; ++j) acc += As[j][c] * va[j];
            double wc = act ? tk * acc : 0.0;
            const double pv = wave_sum(wc * vc);
            const double K = 0.5 * tk * pv;
            wc -= K * vc;
            wa[c] = wc;
            __syncthreads();
#pragma unroll
            for (int j = 0; j < SMALLN; ++j) As[j][c] -= va[j] * wc + wa[j] * vc;
        }
        __syncthreads();
    }
    if (c == 0) d[n - 1] = As[n - 1][n - 1];
    for (int j = 0; j < n; ++j)
        if (cin) A[j * n + c] = As[j][c];
}

// number of eigenvalues of the tridiagonal (d, e) below x
__device__ int sturm(int n, const double* d, const double* e, double x, double pivmin) {
    int cnt = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
    for (int i = 1; i < n; ++i) {
        q = d[i] - x - (e[i - 1] * e[i - 1]) / q;
        if (fabs(q) < pivmin) q = -pivmin;
        if (q < 0) ++cnt;
    }
    return cnt;
}

__device__ void gersh(int n, const double* d, const double* e, double* lo, double* hi, double* tn) {
    double a = INFINITY, b = -INFINITY, c = 0.0;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
        a = fmin(a, d[i] - r);
        b = fmax(b, d[i] + r);
        c = fmax(c, fabs(d[i]) + r);
    }
    *lo = a;
    *hi = b;
    *tn = c;
}

// eigenvalues with indices lo .. lo+cnt-1 (ascending), lo = clamp(count(sigma)
// - nc, 0, n - cnt), cnt = min(2 nc, n); window[0..cnt-1], ctl[0] = lo.
// One wavefront per eigenvalue, by multisection: lane l counts the
// eigenvalues below the point l + 1 of 65 equal steps across the current
// interval, which then shrinks to the step that holds the eigenvalue (six
// bits per round where bisection gains one).  Stops, like bisection, at an
// interval of 2 eps |x| or when the interval no longer shrinks.
__global__ __launch_bounds__(64) void k_bisect_window(int n, const double* dg, const double* eg, double sigma,
                                                      int nc, double* window, int* ctl) {
    // the tridiagonal, read by every Sturm count, staged in LDS
    __shared__ double d[MAXN], e[MAXN];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        d[i] = dg[i];
        e[i] = i + 1 < n ? eg[i] : 0.0;
    }
    __syncthreads();
    const int t = blockIdx.x;
    const int cnt = min(2 * nc, n);
    if (t >= cnt) return;
    const int lane = threadIdx.x;
    double lo, hi, tn;
    gersh(n, d, e, &lo, &hi, &tn);
    const double eps = 2.220446049250313e-16;
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, tn * tn);
    const int i0 = sturm(n, d, e, sigma, pivmin);
    const int first = max(0, min(i0 - nc, n - cnt));
    if (t == 0 && lane == 0) ctl[0] = first;
    const int k = first + t;
    lo -= 2 * eps * tn + 1e-300;
    hi += 2 * eps * tn + 1e-300;
    for (int it = 0; it < 64; ++it) {
        if (hi - lo <= 2 * eps * fmax(fabs(lo), fabs(hi))) break;
        const double w = hi - lo;
        const double x = lo + w * double(lane + 1) / 65.0;
        const unsigned long long above = __ballot(sturm(n, d, e, x, pivmin) >= k + 1);
        double nlo, nhi;
        if (above) {
            const int j = __ffsll(above) - 1;   // first point with the eigenvalue below it
            nhi = lo + w * double(j + 1) / 65.0;
            nlo = j > 0 ? lo + w * double(j) / 65.0 : lo;
        } else {
            nlo = lo + w * 64.0 / 65.0;
            nhi = hi;
        }
        if (!(nlo > lo || nhi < hi)) break;
        lo = nlo;
        hi = nhi;
    }
    if (lane == 0) window[t] = 0.5 * (lo + hi);
}

// the nc window values nearest sigma (ties: the lower value) form a
// contiguous run; theta[0..nc-1] ascending
__global__ void k_pick_window(int n, const double* window, double sigma, int nc, double* theta) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int cnt = min(2 * nc, n);
    int hi = 0;
    while (hi < cnt && window[hi] < sigma) ++hi;
    int lo = hi - 1;
    for (int c = 0; c < nc; ++c) {
        const bool take_lo = lo >= 0 && (hi >= cnt || fabs(window[lo] - sigma) <= fabs(window[hi] - sigma));
        if (take_lo)
            --lo;
        else
            ++hi;
    }
    for (int c = 0; c < nc; ++c) theta[c] = window[lo + 1 + c];
}

// inverse iteration (T - theta_c I) s = b for candidate c: partial-pivot LU
// of the shifted tridiagonal, then three solves from a SplitMix64 start
// vector of the candidate's own.  Element i of the LU arrays and of s sits at
// index i * st of its array (st = 1: the candidate's own scratch; st > 1:
// arrays interleaved over the candidates of a workgroup).
__device__ void invit_one(int n, const double* d, const double* e, double th, int c, double* dd, double* u1,
                          double* u2, double* l, double* piv, double* s, int st) {
    double lo, hi, tn;
    gersh(n, d, e, &lo, &hi, &tn);
    const double tiny = fmax(tn, 1e-300) * 2.220446049250313e-16;
    double dcur = d[0] - th, ucur = n > 1 ? e[0] : 0.0;
    for (int i = 0; i < n - 1; ++i) {
        const double sub = e[i];
        const double dnext = d[i + 1] - th;
        const double unext = i + 2 < n ? e[i + 1] : 0.0;
        if (fabs(dcur) >= fabs(sub)) {
            const double p = fabs(dcur) < tiny ? tiny : dcur;
            const double li = sub / p;
            l[i * st] = li;
            dd[i * st] = p;
            u1[i * st] = ucur;
            u2[i * st] = 0.0;
            piv[i * st] = 0.0;
            dcur = dnext - li * ucur;
            ucur = unext;
        } else {
            const double li = dcur / sub;
            l[i * st] = li;
            dd[i * st] = sub;
            u1[i * st] = dnext;
            u2[i * st] = unext;
            piv[i * st] = 1.0;
            dcur = ucur - li * dnext;
            ucur = -li * unext;
        }
    }
    dd[(n - 1) * st] = fabs(dcur) < tiny ? tiny : dcur;
    for (int i = 0; i < n; ++i) {
        const uint64_t r = splitmix64((uint64_t(c) << 32) + uint64_t(i));
        s[i * st] = double(r >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    }
    for (int it = 0; it < 3; ++it) {
        for (int i = 0; i < n - 1; ++i) {
            if (piv[i * st] != 0.0) {
                const double tt = s[i * st];
                s[i * st] = s[(i + 1) * st];
                s[(i + 1) * st] = tt - l[i * st] * s[i * st];
            } else {
                s[(i + 1) * st] -= l[i * st] * s[i * st];
            }
        }
        s[(n - 1) * st] /= dd[(n - 1) * st];
        if (n > 1) s[(n - 2) * st] = (s[(n - 2) * st] - u1[(n - 2) * st] * s[(n - 1) * st]) / dd[(n - 2) * st];
        for (int i = n - 3; i >= 0; --i)
            s[i * st] = (s[i * st] - u1[i * st] * s[(i + 1) * st] - u2[i * st] * s[(i + 2) * st]) / dd[i * st];
        double nr = 0.0;
        for (int i = 0; i < n; ++i) nr += s[i * st] * s[i * st];
        nr = 1.0 / sqrt(nr);
        for (int i = 0; i < n; ++i) s[i * st] *= nr;
    }
}

// one thread per candidate; work: [nc][5 n] scratch
__global__ void k_invit(int n, const double* d, const double* e, const double* theta, int nc, double* S,
                        double* work) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    double* w = work + int64_t(c) * 5 * n;
    invit_one(n, d, e, theta[c], c, w, w + n, w + 2 * n, w + 3 * n, w + 4 * n, S + int64_t(c) * n, 1);
}

// the same for n <= 64 with the tridiagonal, the LU arrays and the vectors in
// LDS, interleaved over the IC candidates of the workgroup (one thread each)
constexpr int IC = 16;

__global__ __launch_bounds__(IC) void k_invit_lds(int n, const double* dg, const double* eg,
                                                  const double* theta, int nc, double* S) {
    __shared__ double sd[64], se[64];
    __shared__ double lu[5][64][IC], sv[64][IC];
    for (int i = threadIdx.x; i < n; i += IC) {
        sd[i] = dg[i];
        se[i] = i + 1 < n ? eg[i] : 0.0;
    }
    __syncthreads();
    const int j = threadIdx.x, c = blockIdx.x * IC + j;
    if (c >= nc) return;
    invit_one(n, sd, se, theta[c], c, &lu[0][0][j], &lu[1][0][j], &lu[2][0][j], &lu[3][0][j], &lu[4][0][j],
              &sv[0][j], IC);
    for (int i = 0; i < n; ++i) S[int64_t(c) * n + i] = sv[i][j];
}

// Gram-Schmidt (twice) of each candidate against the earlier candidates of
// its cluster (ascending values, consecutive gaps <= 1e-8 |T|); one workgroup
__global__ void k_cluster_orth(int n, const double* d, const double* e, const double* theta, int nc, double* S) {
    __shared__ double sh[17];
    double lo, hi, tn;
    gersh(n, d, e, &lo, &hi, &tn);
    const double ortol = 1e-8 * tn;
    int first = 0;
    for (int c = 0; c < nc; ++c) {
        if (c > 0 && theta[c] - theta[c - 1] > ortol) first = c;
        double* s = S + int64_t(c) * n;
        if (first == c) continue;
        for (int pass = 0; pass < 2; ++pass) {
            for (int q = first; q < c; ++q) {
                const double* o = S + int64_t(q) * n;
                double acc = 0.0;
                for (int i = threadIdx.x; i < n; i += blockDim.x) acc += o[i] * s[i];
                const double dt = wg_sum(acc, sh);
                for (int i = threadIdx.x; i < n; i += blockDim.x) s[i] -= dt * o[i];
                __syncthreads();
            }
        }
        double acc = 0.0;
        for (int i = threadIdx.x; i < n; i += blockDim.x) acc += s[i] * s[i];
        const double inv = 1.0 / sqrt(wg_sum(acc, sh));
        for (int i = threadIdx.x; i < n; i += blockDim.x) s[i] *= inv;
        __syncthreads();
    }
}

// z = H_0 H_1 ... H_{n-2} s for candidate blockIdx.x (in place)
__global__ void k_back_transform(int n, const double* V, const double* tau, double* S) {
    __shared__ double sh[17];
    double* z = S + int64_t(blockIdx.x) * n;
    for (int k = n - 2; k >= 0; --k) {
        const double tk = tau[k];
        if (tk == 0.0) continue;
        const int m = n - k - 1;
        const double* v = V + int64_t(k) * n;
        double acc = 0.0;
        for (int i = threadIdx.x; i < m; i += blockDim.x) acc += v[i] * z[k + 1 + i];
        const double dt = tk * wg_sum(acc, sh);
        for (int i = threadIdx.x; i < m; i += blockDim.x) z[k + 1 + i] -= dt * v[i];
        __syncthreads();
    }
}

}  // namespace

void EigWork::ensure(int n, int nc) {
    const size_t nn = size_t(n) * n;
    V.alloc(nn * 8);
    d.alloc(size_t(n) * 8);
    e.alloc(size_t(n) * 8);
    tau.alloc(size_t(n) * 8);
    window.alloc(size_t(2 * nc + 2) * 8);
    ctl.alloc(64);
    work.alloc(size_t(nc) * 5 * n * 8);
}

void symm_eig_near(hipStream_t st, int n, double* A, double sigma, int nc, EigWork& w, double* theta, double* S) {
    TBH_REQUIRE(n >= 1 && n <= MAXN, "dense eigensolve supports 1 <= n <= 2048");
    TBH_REQUIRE(nc >= 1 && nc <= n, "need 1 <= nc <= n");
    w.ensure(n, nc);
    double* d = w.d.as<double>();
    double* e = w.e.as<double>();
    if (n <= SMALLN)
        hipLaunchKernelGGL(k_sytrd_lds, dim3(1), dim3(64), 0, st, n, A, d, e, w.tau.as<double>(), w.V.as<double>());
    else
        hipLaunchKernelGGL(k_sytrd, dim3(1), dim3(HT), 0, st, n, A, d, e, w.tau.as<double>(), w.V.as<double>());
    const int cnt = std::min(2 * nc, n);
    hipLaunchKernelGGL(k_bisect_window, dim3(cnt), dim3(64), 0, st, n, d, e, sigma, nc, w.window.as<double>(),
                       w.ctl.as<int>());
    hipLaunchKernelGGL(k_pick_window, dim3(1), dim3(64), 0, st, n, w.window.as<double>(), sigma, nc, theta);
    if (n <= SMALLN)
        hipLaunchKernelGGL(k_invit_lds, dim3((nc + IC - 1) / IC), dim3(IC), 0, st, n, d, e, theta, nc, S);
    else
        hipLaunchKernelGGL(k_invit, dim3((nc + 63) / 64), dim3(64), 0, st, n, d, e, theta, nc, S,
                           w.work.as<double>());
    hipLaunchKernelGGL(k_cluster_orth, dim3(1), dim3(256), 0, st, n, d, e, theta, nc, S);
    hipLaunchKernelGGL(k_back_transform, dim3(nc), dim3(256), 0, st, n, w.V.as<double>(), w.tau.as<double>(), S);
    TBH_HIP(hipGetLastError());
}

}  // namespace tbh
