// Dense FP64 symmetric eigensolver (projected matrix of block Lanczos).
#pragma once

#include "tbh_internal.h"

namespace tbh {

struct EigWork {
    DevBuf V, d, e, tau, window, ctl, work;
    void ensure(int n, int nc);
};

// The nc eigenpairs of the symmetric n x n matrix A (device, row-major, both
// triangles; destroyed) whose eigenvalues lie nearest sigma (ties: the lower
// value): theta [nc] ascending and S [nc][n] orthonormal eigenvectors
// (device).  n <= 2048.
void symm_eig_near(hipStream_t st, int n, double* A, double sigma, int nc, EigWork& w, double* theta, double* S);

}  // namespace tbh
