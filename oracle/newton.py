"""Oracle: Newton-Raphson update of the self-consistent potential.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's loop (Sec. III-A, item 3) obtains the converged potential by
Newton-Raphson iteration; it does not say which Jacobian.  The reading
taken here: Newton-Raphson on the self-consistency equation

    G(U) = A U - kappa (n(U) - N_D) = 0,   kappa = 1 / (h^3 eps0 eps_r),

(A = -Lap_h on the grid, U = -phi in eV, n the electrons of the loop's
density rule scattered to the atoms' nodes, N_D the donors), whose root is
the fixed point U_out(U) = U of the loop.  The Jacobian J = A - kappa chi
uses the static density response chi = dn/dU of first-order perturbation
theory over a set S of eigenstates (psi_i, E_i) of H(U):

    chi v = 2 sum_{i,k in S} g_ik rho_ik (rho_ik . v) - 2 d (d . v) / sum_i f'_i,
    rho_ik(j) = sum_alpha psi_i(j, alpha) psi_k(j, alpha)   (pair density on atom j),
    g_ik = (f_i - f_k) / (E_i - E_k),  g_ii = f'_i,   d = sum_i f'_i rho_ii,

for real states; the last term is the Fermi level's shift under charge
neutrality (absent for a given Fermi level).  chi is symmetric and negative
semi-definite, so J is symmetric positive definite.

Readings (the paper is silent on all of them):
* S is the lowest n_states conduction-band-like states (the loop's counted
  states), the response to the rest of the spectrum is left out;
* the occupations inside chi use a smearing temperature kT_J (default
  10 meV) in place of the loop's 4 K: at 4 K the occupations are nearly a
  step in the levels and the linearisation overshoots (measured: a
  two-cycle of the residual at 0.25 eV);
* the Newton steps are accelerated by Anderson mixing of depth m (type II:
  the step d_k = -J^-1 G(U_k) is the residual of the fixed-point map
  U -> U + d), which repairs the Jacobian's remaining error.

Dense linear algebra throughout: the oracle is meant for small slabs.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from oracle import poisson as P
from oracle import scf as S


def neg_laplacian_matrix(grid, h):
    """Sparse A = -Lap_h on [nz, ny, nx] (periodic x, y; Dirichlet z),
    row-major node order (z, y, x)."""
    nx, ny, nz = grid

    def periodic(n):
        m = sp.lil_matrix((n, n))
        for i in range(n):
            m[i, i] += 2.0
            m[i, (i + 1) % n] -= 1.0
            m[i, (i - 1) % n] -= 1.0
        return m.tocsr()

    def dirichlet(n):
        return sp.diags([2.0 * np.ones(n), -np.ones(n - 1), -np.ones(n - 1)], [0, 1, -1], format="csr")

    Ix, Iy, Iz = sp.eye(nx), sp.eye(ny), sp.eye(nz)
    A = sp.kron(dirichlet(nz), sp.kron(Iy, Ix)) + sp.kron(Iz, sp.kron(periodic(ny), Ix)) \
        + sp.kron(Iz, sp.kron(Iy, periodic(nx)))
    return (A / (h * h)).tocsr()


def kappa(h, eps_r):
    return 1.0 / (h ** 3 * P.EPS0_E_PER_V_NM * eps_r)


def pair_densities(psi, n_o):
    """rho[i, k, j] = sum_alpha psi_i(j, alpha) psi_k(j, alpha) for real
    states psi [dim, n_states] (orbital index fastest within an atom)."""
    n_states = psi.shape[1]
    R = np.asarray(psi, dtype=np.float64).reshape(-1, n_o, n_states)
    return np.einsum("jai,jak->ikj", R, R)


def fermi_slope(E, Ef, kT):
    """f'(E) = -f (1 - f) / kT."""
    f = S.occupation(E, Ef, kT)
    return -f * (1.0 - f) / kT


def response_coefficients(E, Ef, kT_J, counted=None):
    """g_ik = (f_i - f_k) / (E_i - E_k) and f'_i, with Fermi-Dirac
    occupations at kT_J.  For levels closer than 1e-5 kT_J (and on the
    diagonal) the divided difference is replaced by the slope at the mean
    level, f'((E_i + E_k) / 2), which it equals to O((E_i - E_k)^2 / kT^2)
    and which does not cancel.  States outside the counted mask (the loop's
    density rule leaves them empty whatever their level) take f = f' = 0."""
    E = np.asarray(E, dtype=np.float64)
    f = S.occupation(E, Ef, kT_J)
    fp = fermi_slope(E, Ef, kT_J)
    cnt = np.ones(E.size, bool) if counted is None else np.asarray(counted, bool)
    f = np.where(cnt, f, 0.0)
    fp = np.where(cnt, fp, 0.0)
    dE = E[:, None] - E[None, :]
    close = np.abs(dE) <= 1e-5 * kT_J
    both = cnt[:, None] & cnt[None, :]
    mid = np.where(both, fermi_slope(0.5 * (E[:, None] + E[None, :]), Ef, kT_J), 0.0)
    g = np.where(close, mid, (f[:, None] - f[None, :]) / np.where(close, 1.0, dE))
    return g, fp


def response_matrix(psi, n_o, E, Ef, kT_J, fixed=False, counted=None):
    """chi [n_atoms, n_atoms] = dn/dU over the states psi (real, unit) with
    levels E; fixed: Fermi level given (no neutrality term); counted: mask
    of the states the density rule fills (default all)."""
    rho = pair_densities(psi, n_o)
    g, fp = response_coefficients(E, Ef, kT_J, counted)
    chi = 2.0 * np.einsum("ik,ikj,ikl->jl", g, rho, rho)
    if not fixed and fp.sum() < 0.0:
        d = np.einsum("i,iij->j", fp, rho)
        chi -= 2.0 * np.outer(d, d) / fp.sum()
    return chi


def newton_step(A, kap, nodes, chi, G):
    """d = -J^-1 G with J = A - kappa P chi P^T (P scatters atoms to nodes)."""
    J = A.toarray()
    J[np.ix_(nodes, nodes)] -= kap * chi
    return np.linalg.solve(J, -G)


def anderson(Xs, Fs):
    """Type II Anderson update from the iterates Xs and their fixed-point
    residuals Fs (oldest first, the newest last): x + f - (dX + dF) gamma
    with gamma the least-squares solution of dF gamma = f."""
    x, f = Xs[-1], Fs[-1]
    if len(Xs) < 2:
        return x + f
    dX = np.stack([Xs[i + 1] - Xs[i] for i in range(len(Xs) - 1)], axis=1)
    dF = np.stack([Fs[i + 1] - Fs[i] for i in range(len(Fs) - 1)], axis=1)
    gamma = np.linalg.lstsq(dF, f, rcond=None)[0]
    return x + f - (dX + dF) @ gamma


def eigenstates(H0, n_o, nodes, U, sigma_mid):
    """Dense eigenpairs of H(U) (ascending) and the mask of the counted
    (conduction-band-like) ones."""
    Ua = np.asarray(U, dtype=np.float64).ravel()[nodes]
    E, psi = np.linalg.eigh(H0 + np.diag(np.repeat(Ua, n_o)))
    wts = S.atom_weights(psi, n_o)
    return E, psi, E - wts @ Ua > sigma_mid


def scf_newton(prob, donors, grid, U0, sigma_mid, tol=1e-4, max_iter=100, T_K=4.0, eps_r=11.7, h_nm=None,
               Ef_fixed=None, cg_tol=1e-12, n_states=64, kT_J=0.01, depth=4, keep_iterates=True, exact=False):
    """The loop with Newton-Raphson (+ Anderson) updates in place of linear
    mixing.  Each step: the loop body at U (its U_out and the stopping
    residual max |U_out - U| are the plain loop's), then the Newton step
    from the n_states lowest counted states and the Anderson update.
    exact: the Jacobian from every eigenstate instead (the counted ones
    filled, the rest empty), i.e. the exact derivative of the density rule
    when kT_J is the loop's temperature.
    Returns dict(U, iterations, residuals, iterates, steps, converged)."""
    from oracle import tb as T
    from workloads import H_GRID_NM
    h = H_GRID_NM if h_nm is None else h_nm
    nx, ny, nz = grid
    kT = S.KB_EV * T_K
    blk = T.build_blocks(prob)
    n_o = blk["n_o"]
    H0 = T.csr_hamiltonian(blk).toarray()
    nodes = S.node_index(prob.pos_q, grid)
    nd = np.zeros(nx * ny * nz)
    np.add.at(nd, nodes[donors], 1.0)
    n_elec = float(len(donors))
    A = neg_laplacian_matrix(grid, h)
    kap = kappa(h, eps_r)
    U = np.array(U0, dtype=np.float64).ravel().copy()
    res_hist, iterates, steps, Xs, Fs = [], [], [], [], []
    converged = False
    for it in range(max_iter):
        o = S.loop_body(H0, n_o, nodes, nd, U.reshape(nz, ny, nx), grid, sigma_mid, n_elec, kT, h, eps_r,
                        Ef_fixed, cg_tol)
        res = float(np.abs(o["U_out"].ravel() - U).max())
        res_hist.append(res)
        if keep_iterates:
            iterates.append(U.reshape(nz, ny, nx).copy())
        if res < tol:
            converged = True
            break
        # G(U) = A U - kappa (n - N_D) = A U + kappa h^3 rho, rho = (N_D - n) / h^3
        G = A @ U + kap * h ** 3 * o["rho"].ravel()
        E, psi, cb = eigenstates(H0, n_o, nodes, U, sigma_mid)
        if exact:
            chi = response_matrix(psi, n_o, E, o["Ef"], kT_J, fixed=Ef_fixed is not None, counted=cb)
        else:
            sel = np.flatnonzero(cb)[:n_states]
            chi = response_matrix(psi[:, sel], n_o, E[sel], o["Ef"], kT_J, fixed=Ef_fixed is not None)
        d = newton_step(A, kap, nodes, chi, G)
        steps.append(d.reshape(nz, ny, nx))
        Xs.append(U.copy())
        Fs.append(d)
        Xs, Fs = Xs[-(depth + 1):], Fs[-(depth + 1):]
        U = anderson(Xs, Fs) if depth > 0 else U + d
    return dict(U=U.reshape(nz, ny, nx), iterations=len(res_hist), residuals=res_hist, iterates=iterates,
                steps=steps, converged=converged)
