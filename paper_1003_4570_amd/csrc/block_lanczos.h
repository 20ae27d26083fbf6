// Block Lanczos internals shared by block_lanczos.hip, the SCF driver and the
// C ABI.
#pragma once

#include "dense_eig.h"
#include "tbh_internal.h"

namespace tbh {

// device workspace of block Lanczos on one ham
struct BlWork {
    int b = 0, mmax = 0;
    int64_t dim = 0;
    DevBuf Q;        // [mmax + 1][dim][b] FP32 basis blocks
    DevBuf W, W2;    // [dim][b] FP32 work blocks
    DevBuf coef;     // FP64: A [mmax][b][b], B [mmax + 1][b][b], C [mmax + 1][b][b], small matrices
    DevBuf part;     // partial sums of the block inner products
    DevBuf T;        // [m b][m b] FP64 projected matrix
    DevBuf theta, S; // [nc], [nc][m b]
    DevBuf Y, Z;     // Ritz vectors [nc][dim] FP64 (state-major), H y [dim] FP64
    DevBuf res;      // [nc][4]: theta, residual, refined, |y|
    DevBuf ctl;      // device control words (deflation count, norms)
    DevBuf mvdesc;   // multi-vector descriptor
    EigWork eig;
    int deflated = 0;     // deflated columns over the last run
    double hx_ms = 0.0;   // H.X time of the last run (when timed)
    // launch shape of the filter's multi-vector products (persistent grid and
    // atom walk), picked by timing the candidates on the first product for
    // a given (H, b); the products do not depend on it
    const void* mv_key = nullptr;
    int64_t mv_n = 0;
    int mv_b = 0, mv_grid = 0, mv_remap = 1;
    void ensure(const Ham& h, int b, int m, int nc);
};

struct BlOpts {
    int b = 32, m = 8, nc = 32;
    double sigma = 0.0;
    double defl_tol = 1e-6;
    bool time_hx = false;
    // operator (H - sigma)^2 instead of H: the pairs nearest sigma become its
    // smallest eigenvalues (extremal, so Rayleigh-Ritz has no spurious
    // values there); each block step applies H twice
    bool fold = false;
};

// One block Lanczos run of m block steps with full reorthogonalisation from
// the start block X0 (device [dim][b] FP32, overwritten), then Rayleigh-Ritz:
// the nc Ritz pairs nearest sigma in W.theta / W.Y, with FP64 residuals and
// Rayleigh quotients in W.res.  Needs the multi-vector copy and the FP64 copy.
void block_lanczos_run(Ham& h, BlWork& W, const BlOpts& o, float* X0);
// Chebyshev-filtered subspace iteration on (H - s)^2 (the self-consistent
// loop's eigen-solve): the block, its filter buffers, and the Ritz pairs
struct FsWork {
    int b = 0;
    int64_t rows = 0;
    DevBuf Y, Y0, Y1, T1, FY;   // [dim][b] FP32 blocks; Y holds the current block
    DevBuf theta, res4;         // [b] Ritz values ascending; [b][4] (theta, residual, theta, |y|)
    DevBuf states;              // [b][dim] FP64 Ritz vectors (state-major, not normalised)
    DevBuf part;
    std::vector<double> last_r4;   // host copy of res4 after the last solve's final Rayleigh-Ritz
    void ensure(int64_t dim, int b);
};

struct FsOpts {
    double s = 0.0;                        // fold centre
    double fmin = 0.0, fcut = 1.0, fmax = 2.0;   // F bounds: wanted >= fmin, damped [fcut, fmax]
    int degree = 20;
};

// F.Y <- p_d((H - s)^2) F.Y, the scaled Chebyshev filter damping [fcut, fmax]
void chfsi_filter(Ham& h, BlWork& W, FsWork& F, const FsOpts& o);
// orthonormalise F.Y and rotate it to the Ritz vectors of H on its span:
// F.theta, F.res4 (residuals from FP32 products, FP64 sums), and with
// states = true the FP64 state-major copy F.states
void chfsi_rayleigh_ritz(Ham& h, BlWork& W, FsWork& F, bool states);
void chfsi_random(hipStream_t st, FsWork& F, uint64_t salt);

// bounds of the spectrum of H (its current potential included): the extreme
// Ritz values of 60 Lanczos steps widened by the last coupling
void spectral_bounds(Ham& h, double* emin, double* emax);

struct FsSolve {
    double s = 0.0;              // fold centre (in the gap)
    double emin = 0.0, emax = 0.0;
    int degree = 20, degree_cold = 60;
    int min_iter = 0, max_iter = 50;
    int k = 1;                   // pairs nearest s that must converge
    double res_tol = 1e-4;
    // warm start only: take the filter's damping bound from the Ritz values
    // the previous solve ended with instead of a Rayleigh-Ritz pass of the
    // start block (for small changes of H between solves)
    bool reuse_ritz = false;
};

// Filter iterations from the current block (warm) or a SplitMix64 block
// until the k Ritz pairs nearest s have residual <= res_tol (at least
// min_iter, at most max_iter); F.states then holds the FP64 states and
// theta_h / res4_h (host, may be null) the Ritz values and [b][4] records.
// Returns the iterations made.
int filtered_solve(Ham& h, BlWork& W, FsWork& F, const FsSolve& o, bool warm, double* theta_h, double* res4_h);

// X [dim][b] FP32 from the FP64 state-major Y [b][dim] (device)
void block_from_states(hipStream_t st, int64_t dim, int b, const double* Y, float* X);
// X [dim][b] FP32 filled with SplitMix64 values in [-1, 1) (stream `salt`)
void block_random(hipStream_t st, int64_t dim, int b, uint64_t salt, float* X);

}  // namespace tbh
