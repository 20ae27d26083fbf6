// Direct solve of the finite-difference Poisson equation of the
// self-consistent loop (Sec. III-A item 3): A x = b with A = -Lap_h on the
// [nz][ny][nx] grid, periodic in x and y, x = 0 on the ghost planes z = -1
// and z = nz.
//
// A is diagonal in the discrete Fourier modes along x and y: mode (kx, ky)
// sees the one-dimensional operator
//     (T x)_z = ((2 + s_x + s_y) x_z - x_{z-1} - x_{z+1}) / h^2,
//     s_x = 2 - 2 cos(2 pi kx / nx),  s_y = 2 - 2 cos(2 pi ky / ny),
// a symmetric positive definite tridiagonal matrix, solved by elimination
// down and back up the column (Thomas).  So: a DFT along x (real input),
// a DFT along y, one tridiagonal solve per (kx, ky) column, and the inverse
// transforms.  The transforms are direct sums (nx, ny <= 64 terms per
// output; the slab grid is 32 x 32), FP64 throughout, fixed order.
//
// The loop uses it in two places: as its Poisson solve (the residual of the
// direct solution is checked, and conjugate gradients take over from it if
// it misses the tolerance), and as the preconditioner of the Newton-Raphson
// Jacobian's conjugate gradients.
#include <cmath>

#include "scf.h"
#include "tbh_internal.h"

namespace tbh {

namespace {

constexpr int TPB = 256;

#define FP_LOOP(i, n) \
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < (n); i += int64_t(gridDim.x) * TPB)

int64_t fp_blocks(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>((n + TPB - 1) / TPB, 4096)); }

// W[z][y][kx] = sum_x b[z][y][x] e^{-2 pi i kx x / nx}   (complex interleaved)
__global__ void k_dft_x(int nx, int ny, int nz, const double* __restrict__ b, const double* __restrict__ cx,
                        const double* __restrict__ sx, double* __restrict__ W) {
    const int64_t n = int64_t(nx) * ny * nz;
    FP_LOOP(i, n) {
        const int kx = int(i % nx);
        const double* row = b + (i - kx);
        double re = 0.0, im = 0.0;
        for (int x = 0; x < nx; ++x) {
            const int t = (kx * x) % nx;
            re += row[x] * cx[t];
            im -= row[x] * sx[t];
        }
        W[2 * i] = re;
        W[2 * i + 1] = im;
    }
}

// V[z][ky][kx] = sum_y W[z][y][kx] e^{sign 2 pi i ky y / ny}
__global__ void k_dft_y(int nx, int ny, int nz, const double* __restrict__ W, const double* __restrict__ cy,
                        const double* __restrict__ sy, double sign, double* __restrict__ V) {
    const int64_t n = int64_t(nx) * ny * nz;
    FP_LOOP(i, n) {
        const int kx = int(i % nx);
        const int ky = int((i / nx) % ny);
        const int64_t plane = i - kx - int64_t(ky) * nx;
        double re = 0.0, im = 0.0;
        for (int y = 0; y < ny; ++y) {
            const int t = (ky * y) % ny;
            const double c = cy[t], s = sign * sy[t];
            const double wr = W[2 * (plane + int64_t(y) * nx + kx)], wi = W[2 * (plane + int64_t(y) * nx + kx) + 1];
            re += wr * c - wi * s;
            im += wr * s + wi * c;
        }
        V[2 * i] = re;
        V[2 * i + 1] = im;
    }
}

// one tridiagonal solve along z per (ky, kx) column, in place on V (complex
// right-hand side, real coefficients); cp holds the eliminated
// super-diagonal of the column
__global__ void k_tridiag_z(int nx, int ny, int nz, double h2, const double* __restrict__ cx,
                            const double* __restrict__ cy, double* __restrict__ V, double* __restrict__ cp) {
    const int64_t cols = int64_t(nx) * ny;
    FP_LOOP(c, cols) {
        const int kx = int(c % nx), ky = int(c / nx);
        const double d = 2.0 + (2.0 - 2.0 * cx[kx]) + (2.0 - 2.0 * cy[ky]);
        // down: y_0 = h^2 v_0 / d, y_z = (h^2 v_z + y_{z-1}) / (d + c'_{z-1}), c'_z = -1 / (d + c'_{z-1})
        double prev = 0.0, yr = 0.0, yi = 0.0;
        for (int z = 0; z < nz; ++z) {
            const int64_t k = int64_t(z) * cols + c;
            const double den = d + prev;
            const double inv = 1.0 / den;
            yr = (h2 * V[2 * k] + yr) * inv;
            yi = (h2 * V[2 * k + 1] + yi) * inv;
            V[2 * k] = yr;
            V[2 * k + 1] = yi;
            prev = -inv;
            cp[k] = prev;
        }
        // up: x_z = y_z - c'_z x_{z+1}
        double xr = 0.0, xi = 0.0;
        for (int z = nz - 1; z >= 0; --z) {
            const int64_t k = int64_t(z) * cols + c;
            xr = V[2 * k] - cp[k] * xr;
            xi = V[2 * k + 1] - cp[k] * xi;
            V[2 * k] = xr;
            V[2 * k + 1] = xi;
        }
    }
}

// x[z][y][x] = Re sum_kx W[z][y][kx] e^{+2 pi i kx x / nx} / (nx ny)
__global__ void k_idft_x(int nx, int ny, int nz, const double* __restrict__ W, const double* __restrict__ cx,
                         const double* __restrict__ sx, double scale, double* __restrict__ out) {
    const int64_t n = int64_t(nx) * ny * nz;
    FP_LOOP(i, n) {
        const int x = int(i % nx);
        const int64_t row = i - x;
        double re = 0.0;
        for (int kx = 0; kx < nx; ++kx) {
            const int t = (kx * x) % nx;
            re += W[2 * (row + kx)] * cx[t] - W[2 * (row + kx) + 1] * sx[t];
        }
        out[i] = re * scale;
    }
}

}  // namespace

void FastPoisson::setup(const int grid[3], double h_nm) {
    if (nx == grid[0] && ny == grid[1] && nz == grid[2] && h == h_nm && W.p) return;
    nx = grid[0];
    ny = grid[1];
    nz = grid[2];
    h = h_nm;
    TBH_REQUIRE(nx >= 1 && ny >= 1 && nz >= 1 && nx <= 4096 && ny <= 4096, "bad Poisson grid");
    const int64_t n = int64_t(nx) * ny * nz;
    W.alloc(size_t(2 * n) * 8);
    V.alloc(size_t(2 * n) * 8);
    cp.alloc(size_t(n) * 8);
    std::vector<double> t(size_t(2 * (nx + ny)));
    for (int k = 0; k < nx; ++k) {
        t[size_t(k)] = std::cos(2.0 * M_PI * k / nx);
        t[size_t(nx + k)] = std::sin(2.0 * M_PI * k / nx);
    }
    for (int k = 0; k < ny; ++k) {
        t[size_t(2 * nx + k)] = std::cos(2.0 * M_PI * k / ny);
        t[size_t(2 * nx + ny + k)] = std::sin(2.0 * M_PI * k / ny);
    }
    tw.alloc(t.size() * 8);
    TBH_HIP(hipMemcpy(tw.p, t.data(), t.size() * 8, hipMemcpyHostToDevice));
}

void FastPoisson::solve(hipStream_t st, const double* b, double* x) {
    const int64_t n = int64_t(nx) * ny * nz;
    const double* cx = tw.as<double>();
    const double* sx = cx + nx;
    const double* cy = cx + 2 * nx;
    const double* sy = cy + ny;
    const int64_t g = fp_blocks(n);
    hipLaunchKernelGGL(k_dft_x, dim3(g), dim3(TPB), 0, st, nx, ny, nz, b, cx, sx, W.as<double>());
    hipLaunchKernelGGL(k_dft_y, dim3(g), dim3(TPB), 0, st, nx, ny, nz, W.as<double>(), cy, sy, -1.0, V.as<double>());
    hipLaunchKernelGGL(k_tridiag_z, dim3(fp_blocks(int64_t(nx) * ny)), dim3(TPB), 0, st, nx, ny, nz, h * h, cx, cy,
                       V.as<double>(), cp.as<double>());
    hipLaunchKernelGGL(k_dft_y, dim3(g), dim3(TPB), 0, st, nx, ny, nz, V.as<double>(), cy, sy, 1.0, W.as<double>());
    hipLaunchKernelGGL(k_idft_x, dim3(g), dim3(TPB), 0, st, nx, ny, nz, W.as<double>(), cx, sx,
                       1.0 / (double(nx) * ny), x);
    TBH_HIP(hipGetLastError());
}

}  // namespace tbh
