// Lanczos solver internals shared by lanczos.hip and the C ABI.
#pragma once

#include "tbh_internal.h"

namespace tbh {

// control slots after alpha[m], beta[m+1]
enum { LZ_TMAX = 0, LZ_BREAK = 2, LZ_STEPS = 3, LZ_INVB = 4, LZ_NCTRL = 8 };   // slot 1 unused

// device view of the scalar state: alpha[j], beta[j] (beta[0] = 0, beta[j]
// couples v_{j-1} and v_j), control slots
struct LzDev {
    double* alpha;
    double* beta;
    double* ctrl;
};

// device workspace of one Lanczos run
struct LzWork {
    DevBuf V, w, scal, part, coef;
    int m = 0;
    int64_t dim = 0;
    bool reorth = false;
    bool full = false;   // V holds every basis vector (needed by reorthogonalisation and by Ritz vectors)
    // captured recurrence, replayed while the key (buffers, m, reorth) holds
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<const void*> key;
    void drop_graph();
    ~LzWork();
    void ensure(const Ham& h, int steps, bool with_reorth, bool keep_basis);
    LzDev dev(int m) const;
};

struct RitzOut {
    DevBuf theta_all, idx, S, work, Y, Z, res;
};

// m steps of the recurrence from the FP64 device start vector v0_dev
// ([dim] scalars, complex interleaved).  Host outputs may be null.  The
// basis V is stored whole when reorthogonalising or when keep_basis is set
// (Ritz vectors need it); otherwise three rotating vectors are kept.
void lanczos_recurrence(Ham& h, LzWork& W, int m, bool reorth, const double* v0_dev, double* alpha_h,
                        double* beta_h, int* steps_h, int* breakdown_h, double* hx_ms, bool keep_basis = false);
void orth_cgs2(Ham& h, LzWork& W, const LzDev& d, int j, hipStream_t st);
// eigenvalues (ascending) of the m x m tridiagonal (FP64 bisection)
void tridiag_gpu(hipStream_t st, int m, const double* alpha_d, const double* beta_d, double* theta_d);
// candidates nearest sigma: Ritz vectors, residuals, Rayleigh quotients;
// out.res = [ncand][4] (theta, residual, refined, |y|).  Needs W.full.
void ritz_pairs(Ham& h, LzWork& W, int steps, double sigma, int ncand, RitzOut& out);
// dst = s * src (FP64, n scalars)
void scale_copy(hipStream_t st, int64_t n, const double* src, double s, double* dst);
void cast_to_f64(hipStream_t st, bool f64, int64_t n, const void* a, double* b);

}  // namespace tbh
