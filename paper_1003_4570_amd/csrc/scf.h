// Schrodinger-Poisson internals shared by scf.hip and the C ABI.
#pragma once

#include "block_lanczos.h"
#include "lanczos.h"
#include "tbh_internal.h"

namespace tbh {

struct PoissonWork {
    DevBuf r, p, Ap, part, s;
    int64_t n = 0;
    void ensure(int64_t n);
};

// device scratch of one CG solve: r, p, Ap [n] FP64; part [2 * 4096]
// block partial sums; s [8] scalar state
struct PoissonBufs {
    double *r, *p, *Ap, *part, *s;
};
constexpr int64_t POISSON_PART = 2 * 4096;
constexpr int64_t POISSON_SCAL = 8;

// FP64 CG for -Lap_h x = b on the grid (periodic x, y; Dirichlet z); x holds
// the initial guess on entry and the solution on exit.
void poisson_cg(hipStream_t st, PoissonWork& W, const int grid[3], double h, const double* b, double* x,
                double rel_tol, int max_iter, int* iters, double* rel_res);
// the same on caller-provided scratch (no allocation)
void poisson_cg_bufs(hipStream_t st, const PoissonBufs& W, const int grid[3], double h, const double* b,
                     double* x, double rel_tol, int max_iter, int* iters, double* rel_res);

// Direct solve of A x = b on the loop's grid (fast_poisson.hip): Fourier
// modes along x and y, one tridiagonal solve along z per mode
struct FastPoisson {
    int nx = 0, ny = 0, nz = 0;
    double h = 0.0;
    DevBuf W, V, cp, tw;
    void setup(const int grid[3], double h_nm);
    void solve(hipStream_t st, const double* b, double* x);   // x may alias b
};

// Newton-Raphson update of the loop's potential (newton.hip)
struct NewtonWork {
    DevBuf R, coef, pairs, sel, inv, fp, diag, d, va, tpart, a, minv, x, r, z, p, Ap, G, Xp, Fp, part, s, small, dX, dF;
    bool have_prev = false;     // an iterate and step are stored for Anderson mixing
    int count = 0, head = 0;    // stored differences, next slot
    std::vector<double> gram;   // dF_l . dF_q of the stored differences
    void reset();
};
struct NewtonIn {
    const double* Y;            // states [.][ns] FP64 (stream order, real)
    int64_t ns;
    int n_o;
    int64_t n_atoms;
    const int64_t* node;        // atom -> grid node (stream order)
    int grid[3];
    double h, kappa;
    const double* b;            // kappa (N_D - n) on the grid
    std::vector<int> sel;       // states of chi (rows of Y), ascending energy
    std::vector<double> E, inv_norm;   // their energies and 1 / |y|
    double Ef, kT;              // Fermi level and the smearing of chi
    bool fixed;                 // Fermi level given (no neutrality term)
    double cg_tol;
    int cg_max_iter;
    int depth;                  // Anderson depth (0 = plain Newton steps)
    FastPoisson* pre;           // preconditioner A^-1 of the Jacobian's CG (null: Jacobi)
};
struct NewtonOut {
    int cg_iters = 0;
    double cg_rel = 0.0;
    int npairs = 0;
};
// one Newton-Raphson step from U (device grid, updated in place)
void newton_update(hipStream_t st, NewtonWork& W, const NewtonIn& in, double* U, NewtonOut* out);

struct Scf {
    Ham* h;
    tbh_scf_opts opt;
    int grid[3];
    int64_t n_nodes = 0;
    int iterations = 0;
    bool have_prev = false;     // a filled state was found on the previous step
    double prev_emin = 0.0;     // lowest filled state energy of the previous step
    DevBuf node_d, b0_d, U, phi, b, Ua, v0, part, occ, q, out, n_atoms_d;
    PoissonWork pw;
    FastPoisson fp;             // the loop's Poisson solve (checked, CG takes over if it misses)
    std::shared_ptr<LzWork> lz;
    RitzOut ritz;
    // start potential (tbh_scf_set_start) and the fallback to the zero start
    DevBuf dmap_d, mask_d, ubare_d, xin_d, xop_d, yop_d, acc_d;
    bool have_ubare = false;
    int start_kind = 0;
    double first_res_limit = 0.0;
    int since_start = 0, grow = 0;
    double prev_res = 0.0;
    void compute_ubare();
    void set_start(const tbh_scf_start& st);
    // filtered subspace eigen-solve (eig_mode 1)
    std::shared_ptr<BlWork> blw;
    std::shared_ptr<FsWork> fs;
    bool fs_warm = false, have_bounds = false;
    bool fs_reuse = false;      // the block's last Ritz values describe the current start
    bool zero_start = true;     // U was set to zero (construction or set_potential(NULL))
    DevBuf U_bounds;            // the potential the spectral bounds were taken at
    double emin_b = 0.0, emax_b = 0.0, last_res = 0.0;
    // Newton-Raphson update (update_mode 1)
    NewtonWork nw;
    Scf(Ham* h, const tbh_scf_opts& o);
    void set_potential(const double* U_dev);
    void step(tbh_scf_report& rep);
};

}  // namespace tbh
