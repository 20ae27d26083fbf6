"""Oracle: finite-difference Poisson equation on the a/4 grid.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's Poisson solver uses finite differences (Sec. III-A, item 3).  The
discretisation here is the standard 7-point Laplacian on the uniform grid
whose nodes are the a/4 lattice points (so every atom sits on a node):

    -eps0 eps_r (Lap_h phi)(r) = rho(r)

periodic in x and y, phi = 0 on the ghost planes z = -1 and z = nz.  Units:
phi in volts, rho in elementary charges per nm^3, h in nm, so
eps0 = 0.0552634936 e / (V nm).  An electron's potential energy is
U = -e phi, i.e. U[eV] = -phi[V].

cg() is textbook conjugate gradients in FP64 on the symmetric positive
definite operator A = -Lap_h; spectral_solve() is an independent exact solve
of the same discrete equations (FFT along x and y, sine transform along z).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

EPS0_E_PER_V_NM = 8.8541878128e-12 / 1.602176634e-19 * 1e-9   # 0.0552634936...
COULOMB_EV_NM = 1.0 / (4.0 * np.pi * EPS0_E_PER_V_NM)          # e^2/(4 pi eps0) = 1.439964 eV nm


def neg_laplacian(phi, h):
    """A phi = -Lap_h phi for phi[nz, ny, nx] (periodic x, y; Dirichlet z)."""
    out = 6.0 * phi
    out -= np.roll(phi, 1, axis=2) + np.roll(phi, -1, axis=2)
    out -= np.roll(phi, 1, axis=1) + np.roll(phi, -1, axis=1)
    out[1:] -= phi[:-1]
    out[:-1] -= phi[1:]
    return out / (h * h)


def rhs(rho, eps_r):
    """Right-hand side b = rho / (eps0 eps_r) of A phi = b."""
    return rho / (EPS0_E_PER_V_NM * eps_r)


def cg(b, h, x0=None, rel_tol=1e-10, max_iter=100000):
    """Conjugate gradients on A x = b.  Returns (x, iterations, rel_residual)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - neg_laplacian(x, h)
    p = r.copy()
    rr = float(np.vdot(r, r))
    bn = float(np.sqrt(np.vdot(b, b)))
    if bn == 0.0:
        return x, 0, 0.0
    it = 0
    while np.sqrt(rr) / bn > rel_tol and it < max_iter:
        Ap = neg_laplacian(p, h)
        alpha = rr / float(np.vdot(p, Ap))
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(np.vdot(r, r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it, float(np.sqrt(rr) / bn)


def spectral_solve(b, h):
    """Exact solve of A x = b: the operator is diagonal in the basis of
    periodic Fourier modes (x, y) times Dirichlet sine modes (z)."""
    nz, ny, nx = b.shape
    kx = 2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(nx) / nx)
    ky = 2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(ny) / ny)
    kz = 2.0 - 2.0 * np.cos(np.pi * np.arange(1, nz + 1) / (nz + 1))
    lam = (kz[:, None, None] + ky[None, :, None] + kx[None, None, :]) / (h * h)
    B = sfft.dst(sfft.fft2(b, axes=(1, 2)), type=1, axis=0)
    X = B / lam
    x = sfft.ifft2(sfft.idst(X, type=1, axis=0), axes=(1, 2))
    return x.real


def potential_energy(rho, h, eps_r, U0=None, rel_tol=1e-10):
    """U = -phi (eV) for the charge density rho (e/nm^3), CG from -U0."""
    x0 = None if U0 is None else -U0
    phi, it, rr = cg(rhs(rho, eps_r), h, x0=x0, rel_tol=rel_tol)
    return -phi, it, rr
