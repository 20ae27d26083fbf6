// Schrodinger-Poisson internals shared by scf.hip and the C ABI.
#pragma once

#include "lanczos.h"
#include "tbh_internal.h"

namespace tbh {

struct PoissonWork {
    DevBuf r, p, Ap, part, s;
    int64_t n = 0;
    void ensure(int64_t n);
};

// FP64 CG for -Lap_h x = b on the grid (periodic x, y; Dirichlet z); x holds
// the initial guess on entry and the solution on exit.
void poisson_cg(hipStream_t st, PoissonWork& W, const int grid[3], double h, const double* b, double* x,
                double rel_tol, int max_iter, int* iters, double* rel_res);

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
    std::shared_ptr<LzWork> lz;
    RitzOut ritz;
    Scf(Ham* h, const tbh_scf_opts& o);
    void set_potential(const double* U_dev);
    void step(tbh_scf_report& rep);
};

}  // namespace tbh
