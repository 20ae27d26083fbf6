// Block Lanczos with full reorthogonalisation on the multi-vector H.X (the
// "(block) Lanczos" eigen-solver of Sec. III-A, item 1).
//
// A block of b orthonormal vectors replaces the single Lanczos vector, so an
// eigenvalue of multiplicity up to b appears with its full multiplicity among
// the Ritz values, and a start block can carry several approximate
// eigenvectors at once (warm starts inside the self-consistent loop).  With
// Q_1 B_0 = X0, for j = 1..m:
//     W = H Q_j - Q_{j-1} B_j^T;  A_j = Q_j^T W;  W -= Q_j A_j;
//     twice { W -= Q (Q^T W) } over Q_1..Q_j;  Q_{j+1} B_{j+1} = W (QR).
// Rayleigh-Ritz on the block-tridiagonal T_m of the A_j and B_j gives Ritz
// pairs; their vectors Y = Q S get explicit FP64 residuals with the FP64
// copy of H.
//
// Precision follows the scalar solver: the basis blocks and H.X are FP32
// (H.X on the matrix cores, 16/32/64 right-hand vectors), every inner
// product, coefficient, the QR's Gram matrices and Cholesky factors, T, its
// eigensolve, the Ritz vectors and residuals are FP64.
//
// Layout: a block is [dim][b] row-major (the multi-vector kernel's X
// layout), the basis [m + 1][dim][b].  Tall-skinny products are two kernels:
// per-chunk partial b x b products (register-tiled, rows staged in LDS) with
// a fixed-order reduction, and a row-parallel update with the small FP64
// coefficient block in LDS.
//
// QR with deflation: Cholesky QR of W (Gram matrix in FP64) run twice; a
// column whose Cholesky pivot is at most defl_tol |H| (the remainder after
// the columns before it is at the FP32 rounding level) is deflated: its row
// of B_{j+1} is zero and its basis vector is a SplitMix64 vector (Steele, Lea
// and Flood, OOPSLA 2014) at counter ((j b + i) << 32) + e, orthogonalised
// against the whole basis.  The replacement directions let the block Krylov
// space grow past an eigenspace of multiplicity above b.
#include <algorithm>
#include <chrono>
#include <cmath>

#include <numeric>
#include <random>

#include "block_lanczos.h"
#include "hx_multi.h"
#include "lanczos.h"

namespace tbh {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double unit_uniform(uint64_t counter) {
    return double(splitmix64(counter) >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < int(blockDim.x >> 6); ++w) r += sh[w];
    __syncthreads();
    return r;
}

// part[chunk][q][k][c] = sum over the chunk's rows r of Q_q[r][k] W[r][c].
// Tiles of RB rows of Q_q and W pass through LDS; while a tile's products
// run, every thread holds its share of the next tile in registers, so the
// loads of one tile overlap the arithmetic of the one before (a chunk is
// swept by one workgroup, often the only one on its compute unit).  Each
// thread accumulates a TR x TC patch in FP64, rows in ascending order.
template <int B>
__global__ __launch_bounds__(TPB) void k_ts_dots(int64_t rows, const float* __restrict__ Q, int64_t qstride,
                                                 int nq, const float* __restrict__ W, int64_t chunk_rows,
                                                 double* __restrict__ part) {
    constexpr int TR = B / 16, TC = B / 16, NCG = B / TC;
    constexpr int RB = 64;
    constexpr int NV = RB * B / 4;                   // float4 per tile and operand
    constexpr int PV = (NV + TPB - 1) / TPB;         // float4 per thread and operand
    __shared__ __align__(16) float qs[RB][B];
    __shared__ __align__(16) float ws[RB][B];
    const int t = threadIdx.x;
    const int tr = t / NCG, tc = t % NCG;
    const int q = blockIdx.y;
    const float* __restrict__ Qb = Q + int64_t(q) * qstride;
    const int64_t r0 = int64_t(blockIdx.x) * chunk_rows;
    const int64_t r1 = r0 + chunk_rows < rows ? r0 + chunk_rows : rows;
    typedef float f4 __attribute__((ext_vector_type(4)));
    f4 pq[PV], pw[PV];
    // element e of a tile starting at row rs: row rs + e / (B / 4), float4 e % (B / 4)
    auto load = [&](int64_t rs) {
        const int nr = int(r1 - rs < RB ? r1 - rs : RB);
#pragma unroll
        for (int p = 0; p < PV; ++p) {
            const int e = t + p * TPB;
            const int rr = e / (B / 4), c4 = e % (B / 4);
            const bool ok = e < NV && rr < nr;
            pq[p] = ok ? *reinterpret_cast<const f4*>(Qb + (rs + rr) * B + 4 * c4) : f4{0.f, 0.f, 0.f, 0.f};
            pw[p] = ok ? *reinterpret_cast<const f4*>(W + (rs + rr) * B + 4 * c4) : f4{0.f, 0.f, 0.f, 0.f};
        }
    };
    double acc[TR][TC];
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TC; ++j) acc[i][j] = 0.0;
    if (r0 < r1) load(r0);
    for (int64_t rs = r0; rs < r1; rs += RB) {
        const int nr = int(r1 - rs < RB ? r1 - rs : RB);
        __syncthreads();
#pragma unroll
        for (int p = 0; p < PV; ++p) {
            const int e = t + p * TPB;
            if (e < NV) {
                reinterpret_cast<f4*>(&qs[0][0])[e] = pq[p];
                reinterpret_cast<f4*>(&ws[0][0])[e] = pw[p];
            }
        }
        __syncthreads();
        if (rs + RB < r1) load(rs + RB);
        auto row = [&](int rr) {
            double qv[TR], wv[TC];
#pragma unroll
            for (int i = 0; i < TR; ++i) qv[i] = double(qs[rr][tr * TR + i]);
#pragma unroll
            for (int j = 0; j < TC; ++j) wv[j] = double(ws[rr][tc * TC + j]);
#pragma unroll
            for (int i = 0; i < TR; ++i)
#pragma unroll
                for (int j = 0; j < TC; ++j) acc[i][j] = fma(qv[i], wv[j], acc[i][j]);
        };
        if (nr == RB) {
#pragma unroll 8
            for (int rr = 0; rr < RB; ++rr) row(rr);
        } else {
            for (int rr = 0; rr < nr; ++rr) row(rr);
        }
    }
    double* out = part + (int64_t(blockIdx.x) * nq + q) * B * B;
#pragma unroll
    for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TC; ++j) out[(tr * TR + i) * B + tc * TC + j] = acc[i][j];
}

// out[i] = sum over chunks of part[chunk][i]: 16 coefficients x 16 slices per
// workgroup, slice s adding chunks s, s + 16, ... in order (loads issued in
// batches), then the slices added in order
__global__ __launch_bounds__(TPB) void k_ts_reduce(int nchunk, int64_t ncoef, const double* __restrict__ part,
                                                   double* __restrict__ out) {
    __shared__ double sh[16][17];
    const int c = threadIdx.x & 15, sl = threadIdx.x >> 4;
    const int64_t i = int64_t(blockIdx.x) * 16 + c;
    double s = 0.0;
    if (i < ncoef) {
        constexpr int BATCH = 8;
        int k = sl;
        for (; k + 16 * (BATCH - 1) < nchunk; k += 16 * BATCH) {
            double v[BATCH];
#pragma unroll
            for (int u = 0; u < BATCH; ++u) v[u] = part[int64_t(k + 16 * u) * ncoef + i];
#pragma unroll
            for (int u = 0; u < BATCH; ++u) s += v[u];
        }
        for (; k < nchunk; k += 16) s += part[int64_t(k) * ncoef + i];
    }
    sh[sl][c] = s;
    __syncthreads();
    if (sl == 0 && i < ncoef) {
        double r = 0.0;
        for (int q = 0; q < 16; ++q) r += sh[q][c];
        out[i] = r;
    }
}

// MODE 0: W[r][c] -= sum_q sum_k Q_q[r][k] C[q][k][c]
// MODE 1: W[r][c]  = sum_k Q_0[r][k] C[0][k][c]        (W and Q distinct)
// The FP64 coefficient block of each q sits in LDS.  A thread owns RPT rows
// x CPT columns (rows rl + i GROUPS of the workgroup's span, so a
// wavefront's rows are adjacent), and every coefficient it reads from LDS
// serves RPT rows.  Per element the sum runs over q, then k, ascending.
template <int B, int MODE>
__global__ __launch_bounds__(TPB) void k_ts_update(int64_t rows, const float* __restrict__ Q, int64_t qstride,
                                                   int nq, const double* __restrict__ C, float* __restrict__ W) {
    constexpr int CPT = 8, TPR = B / CPT, GROUPS = TPB / TPR, RPT = 4, RPB = GROUPS * RPT;
    __shared__ double cs[B * B];
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int t = threadIdx.x;
    const int rl = t / TPR, cg = t % TPR;
    const int64_t rbase = int64_t(blockIdx.x) * RPB + rl;
    double acc[RPT][CPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i)
#pragma unroll
        for (int j = 0; j < CPT; ++j) acc[i][j] = 0.0;
    for (int q = 0; q < nq; ++q) {
        __syncthreads();
        for (int i = t; i < B * B; i += TPB) cs[i] = C[int64_t(q) * B * B + i];
        __syncthreads();
        const float* __restrict__ Qq = Q + int64_t(q) * qstride;
        for (int k0 = 0; k0 < B; k0 += 4) {
            f4 qv[RPT];
#pragma unroll
            for (int i = 0; i < RPT; ++i) {
                const int64_t r = rbase + int64_t(i) * GROUPS;
                qv[i] = r < rows ? *reinterpret_cast<const f4*>(Qq + r * B + k0) : f4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                double cv[CPT];
#pragma unroll
                for (int j = 0; j < CPT; ++j) cv[j] = cs[(k0 + kk) * B + cg * CPT + j];
#pragma unroll
                for (int i = 0; i < RPT; ++i) {
                    const double qk = double(qv[i][kk]);
#pragma unroll
                    for (int j = 0; j < CPT; ++j) acc[i][j] = fma(qk, cv[j], acc[i][j]);
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
        const int64_t r = rbase + int64_t(i) * GROUPS;
        if (r >= rows) continue;
        float* __restrict__ wrow = W + r * B + cg * CPT;
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            if constexpr (MODE == 0)
                wrow[j] = float(double(wrow[j]) - acc[i][j]);
            else
                wrow[j] = float(acc[i][j]);
        }
    }
}

// control words in BlWork::ctl (doubles)
enum { CT_HNORM = 0, CT_NDEFL = 1, CT_NCTL = 8 };

// Cholesky of the Gram matrix G = W^T W with deflation, and the inverse of
// the factor on the kept columns.  One workgroup of 64 threads (b <= 64).
// ref_mode 0: threshold defl_tol * ctl[CT_HNORM]; 1: defl_tol * the largest
// column norm of W (the start block).  ctl[CT_NDEFL] counts deflated columns;
// defl[i] = 1 for a deflated column.
__global__ void k_chol_defl(int b, const double* __restrict__ G, double defl_tol, int ref_mode,
                            double* __restrict__ R, double* __restrict__ Rinv, int* __restrict__ defl,
                            double* __restrict__ ctl) {
    // sR holds G's upper triangle, overwritten row by row by the factor; the
    // inverse is then built column by column into the strictly lower
    // triangle (Rinv[i][j] at sR[j][i], i < j), its diagonal in sDg
    __shared__ double sR[64 * 64];
    __shared__ double sDg[64];
    __shared__ int sdef[64];
    const int t = threadIdx.x;
    for (int i = t; i < b * b; i += blockDim.x) sR[i] = (i % b >= i / b) ? G[i] : 0.0;
    __syncthreads();
    double ref = 0.0;
    if (ref_mode == 1) {
        for (int i = 0; i < b; ++i) ref = fmax(ref, sR[i * b + i]);
        ref = sqrt(ref);
    } else {
        ref = ctl[CT_HNORM];
    }
    const double thr2 = (defl_tol * ref) * (defl_tol * ref);
    // right-looking: once row i of the factor is known, every element (r, c)
    // of the trailing upper triangle subtracts R[i][r] R[i][c] at once, so
    // each element sees the subtractions in the order k = 0, 1, ... as in
    // the row-by-row (left-looking) form
    for (int i = 0; i < b; ++i) {
        const double r2 = sR[i * b + i];
        const bool dropped = !(r2 > thr2);
        const double rii = dropped ? 0.0 : sqrt(r2);
        for (int j = i + 1 + t; j < b; j += blockDim.x) sR[i * b + j] = dropped ? 0.0 : sR[i * b + j] / rii;
        __syncthreads();   // row i is final; every read of its pivot is done
        if (t == 0) {
            sdef[i] = dropped ? 1 : 0;
            sR[i * b + i] = rii;
        }
        // thread c owns column c of the trailing block
        for (int c = i + 1 + t; c < b; c += blockDim.x) {
            const double ric = sR[i * b + c];
#pragma unroll 8
            for (int r = i + 1; r <= c; ++r) sR[r * b + c] -= sR[i * b + r] * ric;
        }
        __syncthreads();
    }
    // the factor goes out
    for (int i = t; i < b * b; i += blockDim.x) R[i] = (i % b >= i / b) ? sR[i] : 0.0;
    // its inverse on the kept columns: column j by back substitution from the
    // bottom, each column by one thread (no column reads another)
    for (int j = t; j < b; j += blockDim.x) {
        const bool dj = sdef[j] != 0;
        sDg[j] = dj ? 0.0 : 1.0 / sR[j * b + j];
        for (int i = j - 1; i >= 0; --i) {
            double v = 0.0;
            if (!dj && !sdef[i]) {
                double s = 0.0;
#pragma unroll 8
                for (int k = i + 1; k < j; ++k) s += sR[i * b + k] * sR[j * b + k];
                s += sR[i * b + j] * sDg[j];
                v = -s / sR[i * b + i];
            }
            sR[j * b + i] = v;
        }
    }
    __syncthreads();
    for (int e = t; e < b * b; e += blockDim.x) {
        const int i = e / b, j = e % b;
        Rinv[e] = i < j ? sR[j * b + i] : (i == j ? sDg[i] : 0.0);
    }
    if (t == 0) {
        int nd = 0;
        for (int i = 0; i < b; ++i) {
            defl[i] = sdef[i];
            nd += sdef[i];
        }
        ctl[CT_NDEFL] = double(nd);
    }
}

// C = A B (b x b); transpose_a: C = A^T B.  One workgroup, both operands
// staged in LDS (A transposed on the way in when asked); C may alias A or B.
__global__ void k_small_mm(int b, const double* A, const double* Bm, double* C, int transpose_a) {
    __shared__ double sA[64 * 64], sB[64 * 64];
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
        const int i = e / b, k = e % b;
        sA[e] = transpose_a ? A[k * b + i] : A[e];
        sB[e] = Bm[e];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
        const int i = e / b, j = e % b;
        double s = 0.0;
        for (int k = 0; k < b; ++k) s += sA[i * b + k] * sB[k * b + j];
        C[e] = s;
    }
}

// Bt = B^T
__global__ void k_small_transpose(int b, const double* Bm, double* Bt) {
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
        const int i = e / b, j = e % b;
        Bt[j * b + i] = Bm[i * b + j];
    }
}

// A = (C + C^T) / 2; ctl[HNORM] = max(ctl[HNORM], max |A|, max |Bprev|)
__global__ void k_sym_block(int b, const double* Cm, double* A, const double* Bprev, double* ctl) {
    __shared__ double sh[4];
    double mx = 0.0;
    for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
        const int i = e / b, j = e % b;
        const double a = 0.5 * (Cm[i * b + j] + Cm[j * b + i]);
        A[e] = a;
        mx = fmax(mx, fabs(a));
        if (Bprev) mx = fmax(mx, fabs(Bprev[e]));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = ctl[CT_HNORM];
        for (int w = 0; w < int(blockDim.x >> 6); ++w) m = fmax(m, sh[w]);
        ctl[CT_HNORM] = m;
    }
}

// deflated columns of the block X get the SplitMix64 replacement values
__global__ void k_defl_fill(int64_t rows, int b, int step, const int* __restrict__ defl, float* __restrict__ X) {
    const int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x;
    if (i >= rows * b) return;
    const int col = int(i % b);
    if (!defl[col]) return;
    const int64_t r = i / b;
    const uint64_t ctr = (uint64_t(int64_t(step) * b + col) << 32) + uint64_t(r);
    X[i] = float(unit_uniform(ctr));
}

// T (n = m b) from the diagonal blocks A_j and sub-diagonal blocks B_{j+1}
__global__ void k_assemble_T(int m, int b, const double* __restrict__ A, const double* __restrict__ Bb,
                             double* __restrict__ T) {
    const int n = m * b;
    const int64_t e = int64_t(blockIdx.x) * TPB + threadIdx.x;
    if (e >= int64_t(n) * n) return;
    const int i = int(e / n), j = int(e % n);
    const int bi = i / b, bj = j / b, ii = i % b, jj = j % b;
    double v = 0.0;
    if (bi == bj)
        v = A[(int64_t(bi) * b + ii) * b + jj];
    else if (bi == bj + 1)      // B_{bi} couples blocks bi-1 and bi: T[bi][bi-1] = B_{bi}
        v = Bb[(int64_t(bi) * b + ii) * b + jj];
    else if (bj == bi + 1)      // T[bi][bi+1] = B_{bi+1}^T
        v = Bb[(int64_t(bj) * b + jj) * b + ii];
    T[e] = v;
}

// Y[c][r] = sum_q sum_k Q_q[r][k] S[c][q b + k]  (FP64 Ritz vectors, state-major)
template <int B, int CG>
__global__ __launch_bounds__(TPB) void k_ritz_block(int64_t rows, const float* __restrict__ Q, int64_t qstride,
                                                    int nq, const double* __restrict__ S, int nc,
                                                    double* __restrict__ Y) {
    const int64_t r = int64_t(blockIdx.x) * TPB + threadIdx.x;
    const int c0 = blockIdx.y * CG;
    if (r >= rows) return;
    const int n = nq * B;
    double acc[CG];
#pragma unroll
    for (int t = 0; t < CG; ++t) acc[t] = 0.0;
    for (int q = 0; q < nq; ++q) {
        const float* __restrict__ qrow = Q + int64_t(q) * qstride + r * B;
        for (int k = 0; k < B; ++k) {
            const double v = double(qrow[k]);
#pragma unroll
            for (int t = 0; t < CG; ++t)
                if (c0 + t < nc) acc[t] = fma(S[int64_t(c0 + t) * n + q * B + k], v, acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < CG; ++t)
        if (c0 + t < nc) Y[int64_t(c0 + t) * rows + r] = acc[t];
}

// X[r][c] = Y[c][r] (FP64 states -> FP32 block)
__global__ void k_states_to_block(int64_t rows, int b, const double* __restrict__ Y, float* __restrict__ X) {
    const int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x;
    if (i >= rows * b) return;
    const int64_t r = i / b;
    const int c = int(i % b);
    X[i] = float(Y[int64_t(c) * rows + r]);
}

__global__ void k_block_random(int64_t rows, int b, uint64_t salt, float* __restrict__ X) {
    const int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x;
    if (i >= rows * b) return;
    const int64_t r = i / b;
    const int c = int(i % b);
    X[i] = float(unit_uniform(salt ^ ((uint64_t(c) << 32) + uint64_t(r))));
}

// partials of |y|^2, y.z, |z - theta y|^2
__global__ void k_bl_resid(int64_t n, const double* __restrict__ y, const double* __restrict__ z,
                           const double* __restrict__ theta, int c, double* __restrict__ part) {
    __shared__ double sh[4];
    const double th = theta[c];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB) {
        const double a = y[i], bz = z[i];
        a0 += a * a;
        a1 += a * bz;
        const double rr = bz - th * a;
        a2 += rr * rr;
    }
    a0 = block_sum(a0, sh);
    a1 = block_sum(a1, sh);
    a2 = block_sum(a2, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x * 3 + 0] = a0;
        part[blockIdx.x * 3 + 1] = a1;
        part[blockIdx.x * 3 + 2] = a2;
    }
}

// out[c] = (theta, residual, Rayleigh quotient, |y|); with use_rq the reported
// value and the residual's shift are the Rayleigh quotient (folded operator:
// theta is then an eigenvalue of (H - sigma)^2, not of H)
__global__ void k_bl_resid_reduce(const double* __restrict__ part, int nblk, const double* __restrict__ theta,
                                  int c, double* __restrict__ out, int use_rq) {
    if (threadIdx.x != 0) return;
    double yy = 0.0, yz = 0.0, rr = 0.0;
    for (int k = 0; k < nblk; ++k) {
        yy += part[3 * k];
        yz += part[3 * k + 1];
        rr += part[3 * k + 2];
    }
    const double rq = yz / yy;
    out[c * 4 + 0] = use_rq ? rq : theta[c];
    // |z - rq y|^2 = |z - theta y|^2 - (rq - theta)^2 |y|^2 (the residual at the Rayleigh quotient)
    out[c * 4 + 1] = use_rq ? sqrt(fmax(rr / yy - (rq - theta[c]) * (rq - theta[c]), 0.0)) : sqrt(rr / yy);
    out[c * 4 + 2] = rq;
    out[c * 4 + 3] = sqrt(yy);
}

int64_t grid1(int64_t n) { return (n + TPB - 1) / TPB; }

// ---------------------------------------------------------------------------
// host helpers (templated on the block size)
// ---------------------------------------------------------------------------

struct TsCtx {
    hipStream_t st;
    int64_t rows;
    int b;
    BlWork* W;
};

// row chunks of a block inner product: up to 768 (three workgroups per CU of
// 256), at most 2048 partial blocks over the nq blocks
int chunks_for(int nq) { return std::max(16, std::min(768, 2048 / std::max(1, nq))); }

// C[q][k][c] = sum_r Q_q[r][k] X[r][c] for q < nq  (C: nq b x b FP64, device)
void ts_dots(const TsCtx& c, const float* Q, int nq, const float* X, double* C) {
    const int nch0 = chunks_for(nq);
    const int64_t chunk = std::max<int64_t>(32, (c.rows + nch0 - 1) / nch0);
    const int nch = int((c.rows + chunk - 1) / chunk);
    const int64_t qs = c.rows * c.b;
    double* part = c.W->part.as<double>();
    dim3 g(nch, nq);
    switch (c.b) {
        case 16: hipLaunchKernelGGL(k_ts_dots<16>, g, dim3(TPB), 0, c.st, c.rows, Q, qs, nq, X, chunk, part); break;
        case 32: hipLaunchKernelGGL(k_ts_dots<32>, g, dim3(TPB), 0, c.st, c.rows, Q, qs, nq, X, chunk, part); break;
        case 64: hipLaunchKernelGGL(k_ts_dots<64>, g, dim3(TPB), 0, c.st, c.rows, Q, qs, nq, X, chunk, part); break;
        default: throw Error(TBH_EINVAL, "block size must be 16, 32 or 64");
    }
    const int64_t ncoef = int64_t(nq) * c.b * c.b;
    hipLaunchKernelGGL(k_ts_reduce, dim3(unsigned((ncoef + 15) / 16)), dim3(TPB), 0, c.st, nch, ncoef, part, C);
}

// MODE 0: X -= sum_q Q_q C_q;  MODE 1: X = Q_0 C_0
template <int MODE>
void ts_update(const TsCtx& c, const float* Q, int nq, const double* C, float* X) {
    const int64_t qs = c.rows * c.b;
    const int rpb = 4 * (TPB / (c.b / 8));   // rows per workgroup: 4 per thread, b / 8 threads per row
    const dim3 g(unsigned((c.rows + rpb - 1) / rpb));
    switch (c.b) {
        case 16: hipLaunchKernelGGL((k_ts_update<16, MODE>), g, dim3(TPB), 0, c.st, c.rows, Q, qs, nq, C, X); break;
        case 32: hipLaunchKernelGGL((k_ts_update<32, MODE>), g, dim3(TPB), 0, c.st, c.rows, Q, qs, nq, C, X); break;
        case 64: hipLaunchKernelGGL((k_ts_update<64, MODE>), g, dim3(TPB), 0, c.st, c.rows, Q, qs, nq, C, X); break;
        default: throw Error(TBH_EINVAL, "block size must be 16, 32 or 64");
    }
}

}  // namespace

void BlWork::ensure(const Ham& h, int b_, int m, int nc) {
    TBH_REQUIRE(b_ == 16 || b_ == 32 || b_ == 64, "block size must be 16, 32 or 64");
    TBH_REQUIRE(m >= 1 && int64_t(m) * b_ <= 2048, "block steps m must satisfy 1 <= m and m * b <= 2048");
    TBH_REQUIRE(nc >= 1 && nc <= m * b_, "candidates must satisfy 1 <= nc <= m b");
    const int64_t rows = h.dim;
    if (b != b_ || mmax < m || dim != rows || !Q.p) {
        b = b_;
        mmax = m;
        dim = rows;
        Q.alloc(size_t(m + 1) * rows * b * 4);
        W.alloc(size_t(rows) * b * 4);
        W2.alloc(size_t(rows) * b * 4);
        // A [m][b][b], B [m+1][b][b], C [m+1][b][b], 8 small b x b matrices
        coef.alloc(size_t(3 * m + 2 + 8) * b * b * 8);
        part.alloc(size_t(2048) * b * b * 8);
        ctl.alloc(64 * 8 + 128 * 4);
    }
    T.alloc(size_t(m) * b * m * b * 8);
    theta.alloc(size_t(nc) * 8);
    S.alloc(size_t(nc) * m * b * 8);
    Y.alloc(size_t(nc) * rows * 8);
    Z.alloc(size_t(rows) * 8);
    res.alloc(size_t(nc) * 4 * 8);
}

void block_from_states(hipStream_t st, int64_t dim, int b, const double* Y, float* X) {
    hipLaunchKernelGGL(k_states_to_block, dim3(grid1(dim * b)), dim3(TPB), 0, st, dim, b, Y, X);
    TBH_HIP(hipGetLastError());
}

void block_random(hipStream_t st, int64_t dim, int b, uint64_t salt, float* X) {
    hipLaunchKernelGGL(k_block_random, dim3(grid1(dim * b)), dim3(TPB), 0, st, dim, b, salt, X);
    TBH_HIP(hipGetLastError());
}

namespace {

// QR of X (orthogonal to the first nprev basis blocks already) into Qout,
// with deflation; Bout = the b x b factor.  Uses W.W2 as scratch.
void qr_block(const TsCtx& c, const float* X, float* Qout, double* Bout, int nprev, int step, double defl_tol,
              int ref_mode, double* small) {
    BlWork& W = *c.W;
    const int b = c.b;
    const size_t bb = size_t(b) * b;
    double* G = small;
    double* R1 = small + bb;
    double* R1i = small + 2 * bb;
    double* R2 = small + 3 * bb;
    double* R2i = small + 4 * bb;
    double* Racc = small + 5 * bb;
    double* Rtmp = small + 6 * bb;
    double* ctl = W.ctl.as<double>();
    int* defl = reinterpret_cast<int*>(ctl + 64);
    int* defl2 = defl + 64;    // flags of the later passes (they deflate only an exactly zero column)
    // pass 1 with deflation
    ts_dots(c, X, 1, X, G);
    hipLaunchKernelGGL(k_chol_defl, dim3(1), dim3(64), 0, c.st, b, G, defl_tol, ref_mode, R1, R1i, defl, ctl);
    ts_update<1>(c, X, 1, R1i, Qout);
    double nd = 0.0;
    TBH_HIP(hipMemcpyAsync(&nd, ctl + CT_NDEFL, 8, hipMemcpyDeviceToHost, c.st));
    TBH_HIP(hipStreamSynchronize(c.st));
    const int ndefl = int(nd);
    W.deflated += ndefl;
    if (ndefl > 0) {
        hipLaunchKernelGGL(k_defl_fill, dim3(grid1(c.rows * b)), dim3(TPB), 0, c.st, c.rows, b, step, defl, Qout);
        if (nprev > 0) {
            double* Cc = W.coef.as<double>() + size_t(2 * W.mmax + 1) * bb;
            for (int pass = 0; pass < 2; ++pass) {
                ts_dots(c, W.Q.as<float>(), nprev, Qout, Cc);
                ts_update<0>(c, W.Q.as<float>(), nprev, Cc, Qout);
            }
        }
    }
    // pass 2 (and 3 after a deflation): plain Cholesky QR
    TBH_HIP(hipMemcpyAsync(Racc, R1, bb * 8, hipMemcpyDeviceToDevice, c.st));
    const int passes = ndefl > 0 ? 2 : 1;
    for (int p = 0; p < passes; ++p) {
        ts_dots(c, Qout, 1, Qout, G);
        hipLaunchKernelGGL(k_chol_defl, dim3(1), dim3(64), 0, c.st, b, G, 0.0, 0, R2, R2i, defl2,
                           ctl + CT_NCTL);
        ts_update<1>(c, Qout, 1, R2i, W.W2.as<float>());
        TBH_HIP(hipMemcpyAsync(Qout, W.W2.p, size_t(c.rows) * b * 4, hipMemcpyDeviceToDevice, c.st));
        hipLaunchKernelGGL(k_small_mm, dim3(1), dim3(256), 0, c.st, b, R2, Racc, Rtmp, 0);
        TBH_HIP(hipMemcpyAsync(Racc, Rtmp, bb * 8, hipMemcpyDeviceToDevice, c.st));
    }
    TBH_HIP(hipMemcpyAsync(Bout, Racc, bb * 8, hipMemcpyDeviceToDevice, c.st));
    TBH_HIP(hipGetLastError());
}

}  // namespace

void block_lanczos_run(Ham& h, BlWork& W, const BlOpts& o, float* X0) {
    TBH_REQUIRE(h.has_mv && h.has_f64, "block Lanczos needs the multi-vector copy and the FP64 copy of H");
    TBH_REQUIRE(!h.cplx_h, "block Lanczos supports real H");
    TBH_REQUIRE(!h.permuted, "block Lanczos needs the caller's atom order (the multi-vector copy keeps it)");
    const int b = o.b, m = o.m, nc = o.nc;
    TBH_REQUIRE(mv_supported(h.n_o, b) || (b == 64 && (h.n_o == 5 || h.n_o == 10)),
                "unsupported block size for this orbital count");
    W.ensure(h, b, m, nc);
    hipStream_t st = h.ctx->stream;
    const TsCtx c{st, h.dim, b, &W};
    const size_t bb = size_t(b) * b;
    double* Acoef = W.coef.as<double>();
    double* Bcoef = Acoef + size_t(W.mmax) * bb;
    double* Ccoef = Bcoef + size_t(W.mmax + 1) * bb;
    double* small = Ccoef + size_t(W.mmax + 1) * bb;
    double* Bt = small + 7 * bb;
    float* Qb = W.Q.as<float>();
    const int64_t qs = h.dim * b;
    W.deflated = 0;
    W.hx_ms = 0.0;
    TBH_HIP(hipMemsetAsync(W.ctl.p, 0, W.ctl.bytes, st));
    // Q_1 B_0 = X0
    qr_block(c, X0, Qb, Bcoef, 0, 0, o.defl_tol, 1, small);
    // descriptors: [j] = (H - shift) Q_j into W (or, folded, into W2), [m] = (H - sigma) W2 into W
    MvDesc d{h.mv_blocks.as<float>(), h.nbr_d.as<int32_t>(), h.has_pot ? h.pot_d.as<double>() : nullptr,
             nullptr, o.fold ? W.W2.as<float>() : W.W.as<float>(), 0, h.n, o.fold ? -o.sigma : 0.0};
    W.mvdesc.alloc(sizeof(MvDesc) * size_t(m + 1));
    std::vector<MvDesc> ds(size_t(m + 1), d);
    for (int j = 0; j < m; ++j) ds[size_t(j)].x = Qb + size_t(j) * qs;
    ds[size_t(m)].x = W.W2.as<float>();
    ds[size_t(m)].y = W.W.as<float>();
    TBH_HIP(hipMemcpyAsync(W.mvdesc.p, ds.data(), sizeof(MvDesc) * ds.size(), hipMemcpyHostToDevice, st));
    int dev = 0;
    TBH_HIP(hipGetDevice(&dev));
    int n_cu = 256;
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    const int grid = int(std::min<int64_t>(int64_t(n_cu) * 32, h.n));   // 32 wavefronts per CU hide the gathers
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (o.time_hx) {
        TBH_HIP(hipEventCreate(&e0));
        TBH_HIP(hipEventCreate(&e1));
    }
    for (int j = 0; j < m; ++j) {
        float* Qj = Qb + size_t(j) * qs;
        float* Wb = W.W.as<float>();
        // W = H Q_j
        if (o.time_hx) TBH_HIP(hipEventRecord(e0, st));
        mv_launch(false, h.n_o, b, W.mvdesc.as<MvDesc>() + j, 1, h.n, grid, 1, st);
        if (o.fold) mv_launch(false, h.n_o, b, W.mvdesc.as<MvDesc>() + m, 1, h.n, grid, 1, st);
        if (o.time_hx) {
            TBH_HIP(hipEventRecord(e1, st));
            TBH_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            TBH_HIP(hipEventElapsedTime(&ms, e0, e1));
            W.hx_ms += ms;
        }
        // W -= Q_{j-1} B_j^T
        if (j > 0) {
            hipLaunchKernelGGL(k_small_transpose, dim3(1), dim3(256), 0, st, b, Bcoef + size_t(j) * bb, Bt);
            ts_update<0>(c, Qj - qs, 1, Bt, Wb);
        }
        // A_j = Q_j^T W; W -= Q_j A_j
        ts_dots(c, Qj, 1, Wb, Ccoef);
        hipLaunchKernelGGL(k_sym_block, dim3(1), dim3(256), 0, st, b, Ccoef, Acoef + size_t(j) * bb,
                           j > 0 ? Bcoef + size_t(j) * bb : nullptr, W.ctl.as<double>());
        ts_update<0>(c, Qj, 1, Ccoef, Wb);
        // full reorthogonalisation: twice over Q_1..Q_j
        for (int pass = 0; pass < 2; ++pass) {
            ts_dots(c, Qb, j + 1, Wb, Ccoef);
            ts_update<0>(c, Qb, j + 1, Ccoef, Wb);
        }
        // Q_{j+1} B_{j+1} = W
        qr_block(c, Wb, Qj + qs, Bcoef + size_t(j + 1) * bb, j + 1, j + 1, o.defl_tol, 0, small);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    // Rayleigh-Ritz
    const int n = m * b;
    hipLaunchKernelGGL(k_assemble_T, dim3(grid1(int64_t(n) * n)), dim3(TPB), 0, st, m, b, Acoef, Bcoef,
                       W.T.as<double>());
    // folded: the Ritz values of (H - sigma)^2 nearest 0 are its smallest
    symm_eig_near(st, n, W.T.as<double>(), o.fold ? 0.0 : o.sigma, nc, W.eig, W.theta.as<double>(),
                  W.S.as<double>());
    constexpr int CG = 8;
    const dim3 gr(unsigned(grid1(h.dim)), unsigned((nc + CG - 1) / CG));
    switch (b) {
        case 16: hipLaunchKernelGGL((k_ritz_block<16, CG>), gr, dim3(TPB), 0, st, h.dim, Qb, qs, m, W.S.as<double>(), nc, W.Y.as<double>()); break;
        case 32: hipLaunchKernelGGL((k_ritz_block<32, CG>), gr, dim3(TPB), 0, st, h.dim, Qb, qs, m, W.S.as<double>(), nc, W.Y.as<double>()); break;
        default: hipLaunchKernelGGL((k_ritz_block<64, CG>), gr, dim3(TPB), 0, st, h.dim, Qb, qs, m, W.S.as<double>(), nc, W.Y.as<double>()); break;
    }
    // FP64 residuals and Rayleigh quotients
    const int64_t gres = std::min<int64_t>(1024, grid1(h.dim));
    double* part = W.part.as<double>();
    for (int cnd = 0; cnd < nc; ++cnd) {
        double* y = W.Y.as<double>() + size_t(cnd) * h.dim;
        HxArgs a;
        a.blocks = h.prec == TBH_F64 ? h.blocks.p : h.blocks64.p;
        a.keys = h.keys_d.as<uint8_t>();
        a.nbr = h.nbr_d.as<int32_t>();
        a.x = y;
        a.y = W.Z.p;
        a.pot = h.has_pot ? h.pot_d.as<double>() : nullptr;
        a.n_atoms = h.n;
        hx_launch(h.prec == TBH_F64 ? h.lay : h.lay64, true, a, st);
        hipLaunchKernelGGL(k_bl_resid, dim3(gres), dim3(TPB), 0, st, h.dim, y, W.Z.as<double>(),
                           W.theta.as<double>(), cnd, part);
        hipLaunchKernelGGL(k_bl_resid_reduce, dim3(1), dim3(64), 0, st, part, int(gres), W.theta.as<double>(), cnd,
                           W.res.as<double>(), int(o.fold));
    }
    TBH_HIP(hipGetLastError());
}


// ---------------------------------------------------------------------------
// Chebyshev-filtered subspace iteration on the folded operator (the
// eigen-solve inside the self-consistent loop).
//
// The states the loop fills are the lowest conduction states, which lie
// inside the spectrum (the valence band is below the gap).  With
// F = (H - s)^2 and s in the gap, nearer the conduction band than the
// valence band, they are the smallest eigenvalues of F.  A block Y of b
// vectors is filtered with the scaled Chebyshev polynomial of degree d that
// damps F on [f_cut, f_max] (f_cut the largest F value the block currently
// represents, f_max a bound on F over the spectrum), orthonormalised
// (Cholesky QR), and rotated by the Rayleigh-Ritz of H on its span (Zhou,
// Saad, Tiago and Chelikowsky, J. Comput. Phys. 219 (2006) 172, with the
// scaled three-term recurrence of Zhou and Saad, SIAM J. Matrix Anal. Appl.
// 29 (2007) 954).  Warm-started from the previous step's block, one filter of
// low degree per step keeps pace with the loop.  Only H.X (two shifted
// multi-vector launches per degree), FP32 block storage, FP64 Gram /
// Rayleigh-Ritz matrices and residual sums.
// ---------------------------------------------------------------------------

namespace {

// Y2 = a FY + b Y1 + c Y0
__global__ void k_cheb_combine(int64_t n, const float* __restrict__ FY, const float* __restrict__ Y1,
                               const float* __restrict__ Y0, double a, double b, double c, float* __restrict__ Y2) {
    const int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x;
    if (i >= n) return;
    double v = a * double(FY[i]) + b * double(Y1[i]);
    if (Y0) v += c * double(Y0[i]);
    Y2[i] = float(v);
}

// part[chunk][c] = sum over the chunk's rows of (A[r][c] - theta_c X[r][c])^2
// (theta null: of A[r][c]^2); 256 threads = 4 row lanes x 64 columns
__global__ __launch_bounds__(TPB) void k_col_sq(int64_t rows, int b, const float* __restrict__ A,
                                                const float* __restrict__ X, const double* __restrict__ theta,
                                                int64_t chunk_rows, double* __restrict__ part) {
    __shared__ double sh[TPB];
    const int c = threadIdx.x % 64, lane = threadIdx.x / 64;
    double acc = 0.0;
    if (c < b) {
        const double th = theta ? theta[c] : 0.0;
        const int64_t r0 = int64_t(blockIdx.x) * chunk_rows;
        const int64_t r1 = r0 + chunk_rows < rows ? r0 + chunk_rows : rows;
        for (int64_t r = r0 + lane; r < r1; r += 4) {
            const double v = double(A[r * b + c]) - (X ? th * double(X[r * b + c]) : 0.0);
            acc += v * v;
        }
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (lane == 0 && c < b)
        part[int64_t(blockIdx.x) * b + c] = (sh[c] + sh[64 + c]) + (sh[128 + c] + sh[192 + c]);
}

// res4[c] = (theta, residual, theta, |y|) from the two column sums.  64
// columns x 16 slices: slice s adds chunks s, s + 16, ... in order, then
// the slices are added in order.
__global__ __launch_bounds__(1024) void k_fs_res(int nchunk, int b, const double* __restrict__ pr,
                                                 const double* __restrict__ pn, const double* __restrict__ theta,
                                                 double* __restrict__ res4) {
    __shared__ double sr[16][64], sy[16][64];
    const int c = threadIdx.x & 63, sl = threadIdx.x >> 6;
    double r = 0.0, y = 0.0;
    if (c < b)
        for (int k = sl; k < nchunk; k += 16) {
            r += pr[int64_t(k) * b + c];
            y += pn[int64_t(k) * b + c];
        }
    sr[sl][c] = r;
    sy[sl][c] = y;
    __syncthreads();
    if (sl != 0 || c >= b) return;
    r = 0.0;
    y = 0.0;
    for (int k = 0; k < 16; ++k) {
        r += sr[k][c];
        y += sy[k][c];
    }
    const double yn = sqrt(y);
    res4[4 * c + 0] = theta[c];
    res4[4 * c + 1] = sqrt(r) / yn;
    res4[4 * c + 2] = theta[c];
    res4[4 * c + 3] = yn;
}

// Ys[c][r] = X[r][c] (FP32 block -> FP64 states)
__global__ void k_block_to_states(int64_t rows, int b, const float* __restrict__ X, double* __restrict__ Ys) {
    const int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x;
    if (i >= rows * b) return;
    const int64_t r = i / b;
    const int c = int(i % b);
    Ys[int64_t(c) * rows + r] = double(X[i]);
}

}  // namespace

void FsWork::ensure(int64_t dim, int b_) {
    if (b == b_ && rows == dim && Y.p) return;
    b = b_;
    rows = dim;
    const size_t blk = size_t(dim) * b * 4;
    Y.alloc(blk);
    Y0.alloc(blk);
    Y1.alloc(blk);
    T1.alloc(blk);
    FY.alloc(blk);
    theta.alloc(size_t(b) * 8);
    res4.alloc(size_t(b) * 4 * 8);
    states.alloc(size_t(b) * dim * 8);
    part.alloc(size_t(2) * 1024 * b * 8);
}

namespace {

// the fastest (grid, atom walk) for H.X of this H with b vectors: 4 to 32
// one-wavefront workgroups per compute unit x the three walks, each timed
// over 3 launches after one untimed launch (on the caller's buffers; the
// product that follows overwrites the output)
void tune_mv(Ham& h, BlWork& W, const MvDesc* dd, int b, hipStream_t st) {
    int dev = 0;
    TBH_HIP(hipGetDevice(&dev));
    int n_cu = 256;
    (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TBH_HIP(hipEventCreate(&e0));
    TBH_HIP(hipEventCreate(&e1));
    float best = INFINITY;
    int bg = int(std::min<int64_t>(int64_t(n_cu) * 32, h.n)), br = 1;
    for (int mult : {4, 8, 12, 16, 32})
        for (int remap = 0; remap <= 2; ++remap) {
            const int grid = int(std::max<int64_t>(1, std::min<int64_t>(int64_t(n_cu) * mult, h.n)));
            mv_launch(false, h.n_o, b, dd, 1, h.n, grid, remap, st);
            TBH_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < 3; ++r) mv_launch(false, h.n_o, b, dd, 1, h.n, grid, remap, st);
            TBH_HIP(hipEventRecord(e1, st));
            TBH_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            TBH_HIP(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                bg = grid;
                br = remap;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    W.mv_key = h.mv_blocks.p;
    W.mv_n = h.n;
    W.mv_b = b;
    W.mv_grid = bg;
    W.mv_remap = br;
}

MvDesc mv_desc(Ham& h, const float* in, float* out, double shift) {
    return MvDesc{h.mv_blocks.as<float>(), h.nbr_d.as<int32_t>(), h.has_pot ? h.pot_d.as<double>() : nullptr,
                  in, out, 0, h.n, shift};
}

// the multi-vector product of descriptor slot `slot` of W.mvdesc, in the
// tuned launch shape
void mv_run(Ham& h, BlWork& W, int slot, int b, hipStream_t st) {
    const MvDesc* dd = W.mvdesc.as<MvDesc>() + slot;
    if (W.mv_grid == 0 || W.mv_key != h.mv_blocks.p || W.mv_n != h.n || W.mv_b != b) tune_mv(h, W, dd, b, st);
    mv_launch(false, h.n_o, b, dd, 1, h.n, W.mv_grid, W.mv_remap, st);
}

// one multi-vector launch out = (H + shift) in, its descriptor written to slot `slot`
void mv_apply(Ham& h, BlWork& W, int slot, const float* in, float* out, double shift, int b, hipStream_t st) {
    const MvDesc d = mv_desc(h, in, out, shift);
    TBH_HIP(hipMemcpyAsync(W.mvdesc.as<MvDesc>() + slot, &d, sizeof(d), hipMemcpyHostToDevice, st));
    mv_run(h, W, slot, b, st);
}

}  // namespace

void chfsi_filter(Ham& h, BlWork& W, FsWork& F, const FsOpts& o) {
    TBH_REQUIRE(h.has_mv && !h.cplx_h && !h.permuted, "the filter needs the real multi-vector copy");
    TBH_REQUIRE(o.fmax > o.fcut && o.fcut > o.fmin, "need fmin < fcut < fmax");
    hipStream_t st = h.ctx->stream;
    const int b = F.b;
    const int64_t ne = h.dim * b;
    const double e = 0.5 * (o.fmax - o.fcut), c = 0.5 * (o.fmax + o.fcut);
    double sig = e / (c - o.fmin);
    const double tau = 2.0 / sig;
    // the three blocks of the recurrence rotate; Y0, Y1, Y2 index them
    float* blk[3] = {F.Y.as<float>(), F.Y0.as<float>(), F.Y1.as<float>()};
    int Y0 = 0, Y1 = 1, Y2 = 2;
    float* T1 = F.T1.as<float>();
    float* FY = F.FY.as<float>();
    // descriptors of the call, written once: slot r = (H - s) blk[r] -> T1,
    // slot 3 = (H - s) T1 -> FY
    W.mvdesc.alloc(sizeof(MvDesc) * 8);
    const MvDesc ds[4] = {mv_desc(h, blk[0], T1, -o.s), mv_desc(h, blk[1], T1, -o.s), mv_desc(h, blk[2], T1, -o.s),
                          mv_desc(h, T1, FY, -o.s)};
    TBH_HIP(hipMemcpyAsync(W.mvdesc.p, ds, sizeof(ds), hipMemcpyHostToDevice, st));
    const dim3 g(unsigned((ne + TPB - 1) / TPB));
    // F Y = (H - s)((H - s) Y)
    auto applyF = [&](int in) {
        mv_run(h, W, in, b, st);
        mv_run(h, W, 3, b, st);
    };
    // Y1 = (F Y0 - c Y0) sig / e
    applyF(Y0);
    hipLaunchKernelGGL(k_cheb_combine, g, dim3(TPB), 0, st, ne, FY, blk[Y0], (const float*)nullptr, sig / e,
                       -c * sig / e, 0.0, blk[Y1]);
    for (int i = 2; i <= o.degree; ++i) {
        const double sig2 = 1.0 / (tau - sig);
        applyF(Y1);
        // Y2 = 2 sig2 / e (F Y1 - c Y1) - sig sig2 Y0
        hipLaunchKernelGGL(k_cheb_combine, g, dim3(TPB), 0, st, ne, FY, blk[Y1], blk[Y0], 2.0 * sig2 / e,
                           -2.0 * sig2 * c / e, -sig * sig2, blk[Y2]);
        const int t = Y0;
        Y0 = Y1;
        Y1 = Y2;
        Y2 = t;
        sig = sig2;
    }
    // the filtered block ends in Y1; keep it in F.Y
    if (Y1 != 0)
        TBH_HIP(hipMemcpyAsync(F.Y.p, blk[Y1], size_t(ne) * 4, hipMemcpyDeviceToDevice, st));
    TBH_HIP(hipGetLastError());
}

void chfsi_rayleigh_ritz(Ham& h, BlWork& W, FsWork& F, bool states) {
    hipStream_t st = h.ctx->stream;
    const int b = F.b;
    W.ensure(h, b, 1, b);
    const TsCtx c{st, h.dim, b, &W};
    const size_t bb = size_t(b) * b;
    double* Acoef = W.coef.as<double>();
    double* Ccoef = Acoef + size_t(W.mmax) * bb + size_t(W.mmax + 1) * bb;
    double* small = Ccoef + size_t(W.mmax + 1) * bb;
    double* Bt = small + 7 * bb;
    float* Yq = F.Y0.as<float>();
    float* HY = F.T1.as<float>();
    float* Yr = F.Y.as<float>();
    float* HYr = F.FY.as<float>();
    W.mvdesc.alloc(sizeof(MvDesc) * 8);
    TBH_HIP(hipMemsetAsync(W.ctl.p, 0, W.ctl.bytes, st));
    // orthonormal basis of the filtered block
    qr_block(c, F.Y.as<float>(), Yq, Bt, 0, 0, 1e-6, 1, small);
    // Rayleigh-Ritz of H on its span
    mv_apply(h, W, 4, Yq, HY, 0.0, b, st);
    ts_dots(c, Yq, 1, HY, Ccoef);
    hipLaunchKernelGGL(k_sym_block, dim3(1), dim3(256), 0, st, b, Ccoef, Acoef, (const double*)nullptr,
                       W.ctl.as<double>());
    W.T.alloc(bb * 8);
    W.S.alloc(bb * 8);
    symm_eig_near(st, b, Acoef, 0.0, b, W.eig, F.theta.as<double>(), W.S.as<double>());
    hipLaunchKernelGGL(k_small_transpose, dim3(1), dim3(256), 0, st, b, W.S.as<double>(), Bt);
    ts_update<1>(c, Yq, 1, Bt, Yr);
    ts_update<1>(c, HY, 1, Bt, HYr);
    // residuals |H y - theta y| / |y| from the rotated products
    const int64_t chunk = std::max<int64_t>(256, (h.dim + 1023) / 1024);
    const int nch = int((h.dim + chunk - 1) / chunk);
    double* pr = F.part.as<double>();
    double* pn = pr + size_t(1024) * b;
    hipLaunchKernelGGL(k_col_sq, dim3(nch), dim3(TPB), 0, st, h.dim, b, HYr, Yr, F.theta.as<double>(), chunk, pr);
    hipLaunchKernelGGL(k_col_sq, dim3(nch), dim3(TPB), 0, st, h.dim, b, Yr, (const float*)nullptr,
                       (const double*)nullptr, chunk, pn);
    hipLaunchKernelGGL(k_fs_res, dim3(1), dim3(1024), 0, st, nch, b, pr, pn, F.theta.as<double>(), F.res4.as<double>());
    if (states)
        hipLaunchKernelGGL(k_block_to_states, dim3(unsigned((h.dim * b + TPB - 1) / TPB)), dim3(TPB), 0, st, h.dim,
                           b, Yr, F.states.as<double>());
    TBH_HIP(hipGetLastError());
}

void chfsi_random(hipStream_t st, FsWork& F, uint64_t salt) {
    block_random(st, F.rows, F.b, salt, F.Y.as<float>());
}


void spectral_bounds(Ham& h, double* emin, double* emax) {
    hipStream_t st = h.ctx->stream;
    const int m = 60;
    const size_t ns = size_t(h.dim) * (h.cplx_h ? 2 : 1);
    // a fixed start vector (deterministic), uniform in [-1, 1)
    std::vector<double> v0(ns);
    std::mt19937_64 gen(0x5b0d5ull);
    for (auto& v : v0) v = double(gen() >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    DevBuf v0d, th;
    v0d.alloc(ns * 8);
    TBH_HIP(hipMemcpyAsync(v0d.p, v0.data(), ns * 8, hipMemcpyHostToDevice, st));
    LzWork W;
    std::vector<double> a(m), bt(m);
    int steps = 0, brk = 0;
    lanczos_recurrence(h, W, m, false, v0d.as<double>(), a.data(), bt.data(), &steps, &brk, nullptr, false);
    TBH_REQUIRE(steps >= 2, "spectral bounds: Lanczos made fewer than 2 steps");
    th.alloc(size_t(steps) * 8);
    const LzDev d = W.dev(m);
    tridiag_gpu(st, steps, d.alpha, d.beta, th.as<double>());
    std::vector<double> t(static_cast<size_t>(steps));
    TBH_HIP(hipMemcpyAsync(t.data(), th.p, t.size() * 8, hipMemcpyDeviceToHost, st));
    TBH_HIP(hipStreamSynchronize(st));
    // the extreme Ritz values move outwards by at most the last coupling
    const double last = std::fabs(bt[size_t(steps - 1)]);
    *emin = t.front() - last;
    *emax = t.back() + last;
}

int filtered_solve(Ham& h, BlWork& W, FsWork& F, const FsSolve& o, bool warm, double* theta_h, double* res4_h) {
    hipStream_t st = h.ctx->stream;
    const int b = F.b;
    TBH_REQUIRE(o.k >= 1 && o.k <= b, "k must satisfy 1 <= k <= block");
    if (!warm) chfsi_random(st, F, 0x5eedf11e7ull);
    std::vector<double> r4(size_t(b) * 4);
    auto rr = [&](bool states) {
        chfsi_rayleigh_ritz(h, W, F, states);
        TBH_HIP(hipMemcpyAsync(r4.data(), F.res4.p, r4.size() * 8, hipMemcpyDeviceToHost, st));
        TBH_HIP(hipStreamSynchronize(st));
    };
    // the k Ritz pairs nearest the fold centre (ties: lower value)
    std::vector<int> order(static_cast<size_t>(b));
    auto converged = [&]() {
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            const double dx = std::fabs(r4[4 * x] - o.s), dy = std::fabs(r4[4 * y] - o.s);
            return dx != dy ? dx < dy : r4[4 * x] < r4[4 * y];
        });
        for (int t = 0; t < o.k; ++t)
            if (!(r4[4 * order[size_t(t)] + 1] <= o.res_tol)) return false;
        return true;
    };
    if (warm && o.reuse_ritz && F.last_r4.size() == r4.size() && o.min_iter >= 1)
        r4 = F.last_r4;
    else
        rr(false);
    const double fmax = std::max((o.emax - o.s) * (o.emax - o.s), (o.emin - o.s) * (o.emin - o.s));
    int it = 0;
    while (it < o.max_iter && (it < o.min_iter || !converged())) {
        // damp everything above the largest F value the block represents
        double fcut = 0.0;
        for (int c = 0; c < b; ++c) fcut = std::max(fcut, (r4[4 * c] - o.s) * (r4[4 * c] - o.s));
        fcut = std::min(fcut, 0.5 * fmax);
        FsOpts fo;
        fo.s = o.s;
        fo.fmin = 0.0;
        fo.fcut = std::max(fcut, 1e-6 * fmax);
        fo.fmax = fmax;
        fo.degree = warm || it > 0 ? o.degree : o.degree_cold;
        chfsi_filter(h, W, F, fo);
        rr(false);
        ++it;
    }
    // final pass for the states
    hipLaunchKernelGGL(k_block_to_states, dim3(unsigned((h.dim * b + TPB - 1) / TPB)), dim3(TPB), 0, st, h.dim, b,
                       F.Y.as<float>(), F.states.as<double>());
    TBH_HIP(hipGetLastError());
    F.last_r4 = r4;
    if (theta_h) for (int c = 0; c < b; ++c) theta_h[c] = r4[4 * c];
    if (res4_h) std::copy(r4.begin(), r4.end(), res4_h);
    return it;
}

}  // namespace tbh
