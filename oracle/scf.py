"""Oracle: charge from eigenstates and the self-consistent Schrodinger-Poisson loop.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's self-consistent loop (Sec. III-A) has three parts: eigenstates
of the tight-binding Hamiltonian on the current potential, the charge from
filling those states -- either up to a given Fermi level or with the Fermi
level fixed by charge neutrality -- and a finite-difference Poisson solve
whose potential updates the Hamiltonian; the steps repeat until the
potential is self-consistent.  The application is a P delta layer in Si at
4 K (Sec. III-B).

Readings used where the paper is silent:
* donors are +e point charges on their atoms' grid nodes, electrons sit on
  atom nodes with weight sum_alpha |psi(i, alpha)|^2, spin degeneracy 2;
* only conduction-band-like states count: E_n - <psi_n|U|psi_n> > sigma_mid
  (the gap centre of the bulk bands);
* Fermi-Dirac occupation, E_F by bisection so that 2 sum_n f(E_n) = N_D;
* the update is linear mixing U <- U + alpha (U_out - U) (in place of the
  paper's Newton-Raphson), stopping when max |U_out - U| < tol.

This module's eigen-solve is dense (numpy eigh): the oracle is meant for
small slabs.
"""
from __future__ import annotations

import numpy as np
from scipy.special import expit

from oracle import poisson as P
from oracle import tb as T

KB_EV = 8.617333262e-5


def occupation(E, Ef, kT):
    """Fermi-Dirac f(E) (kT > 0) or the step function (kT == 0)."""
    E = np.asarray(E, dtype=np.float64)
    if kT == 0.0:
        return (E < Ef).astype(np.float64) + 0.5 * (E == Ef)
    return expit(-(E - Ef) / kT)


def fermi_level(E, n_elec, kT, spin_deg=2.0, tol=1e-13):
    """E_F with spin_deg * sum f(E_n) = n_elec, by bisection."""
    E = np.asarray(E, dtype=np.float64)
    if n_elec > spin_deg * E.size:
        raise ValueError("not enough states for the electron count")
    if kT == 0.0:
        # zero temperature: midway between the last filled and first empty level
        Es = np.sort(E)
        nf = n_elec / spin_deg
        k = int(np.floor(nf))
        if nf == k:
            return 0.5 * (Es[k - 1] + Es[k]) if 0 < k < Es.size else Es[min(k, Es.size - 1)]
        return Es[k]
    lo = E.min() - 60 * kT - 1.0
    hi = E.max() + 60 * kT + 1.0
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if spin_deg * occupation(E, mid, kT).sum() < n_elec:
            lo = mid
        else:
            hi = mid
        if hi - lo < tol:
            break
    return 0.5 * (lo + hi)


def atom_weights(psi, n_o):
    """|psi_n(i)|^2 summed over the orbitals of atom i: [n_states, N]."""
    p = np.asarray(psi)
    n_states = p.shape[1]
    return (np.abs(p) ** 2).T.reshape(n_states, -1, n_o).sum(axis=2)


def node_index(pos_q, grid):
    nx, ny, nz = grid
    q = np.asarray(pos_q, dtype=np.int64)
    return (q[:, 2] * ny + q[:, 1]) * nx + q[:, 0]


def electron_density(E, wts, Ua, sigma_mid, n_elec, kT, Ef=None):
    """Electrons per atom from the CB-like states; E_F from neutrality unless
    given.  Returns (n_i, E_F, mask of counted states)."""
    cb = E - wts @ Ua > sigma_mid
    Ec = E[cb]
    if Ef is None:
        Ef = fermi_level(Ec, n_elec, kT)
    f = occupation(Ec, Ef, kT)
    n = 2.0 * (f[:, None] * wts[cb]).sum(axis=0)
    return n, Ef, cb


def loop_body(H0, n_o, nodes, nd, U, grid, sigma_mid, n_elec, kT, h, eps_r, Ef_fixed, cg_tol):
    """One pass of the loop body at input potential U [nz, ny, nx] (eV):
    eigenstates of H(U) = H_TB + U at every orbital of each atom, electrons
    per atom from the CB-like states, rho = e (N_D - n) / h^3 at the atom
    nodes, and U_out = -phi from the Poisson equation (CG started from -U).
    Returns dict(U_out, rho, Ef, n)."""
    nx, ny, nz = grid
    Ua = U.ravel()[nodes]
    Hm = H0 + np.diag(np.repeat(Ua, n_o))
    E, psi = np.linalg.eigh(Hm)
    wts = atom_weights(psi, n_o)
    n_i, Ef, _ = electron_density(E, wts, Ua, sigma_mid, n_elec, kT, Ef_fixed)
    rho = nd.copy()
    np.add.at(rho, nodes, -n_i)
    rho = (rho / h ** 3).reshape(nz, ny, nx)
    Uout, _, _ = P.potential_energy(rho, h, eps_r, U0=U, rel_tol=cg_tol)
    return dict(U_out=Uout, rho=rho, Ef=Ef, n=n_i)


def scf(prob, donors, grid, U0, sigma_mid, alpha=0.1, tol=1e-4, max_iter=200, T_K=4.0,
        eps_r=11.7, h_nm=None, Ef_fixed=None, cg_tol=1e-12, keep_iterates=True):
    """Self-consistent loop with dense eigenstates.  U0: [nz, ny, nx] (eV).
    Returns dict(U, iterations, residuals, iterates, rhos, outputs, Ef,
    converged): iterates[t] is the input potential of step t, rhos[t] and
    outputs[t] its charge density and U_out (kept with keep_iterates)."""
    from workloads import H_GRID_NM
    h = H_GRID_NM if h_nm is None else h_nm
    nx, ny, nz = grid
    kT = KB_EV * T_K
    blk = T.build_blocks(prob)
    n_o = blk["n_o"]
    H0 = T.csr_hamiltonian(blk).toarray()
    nodes = node_index(prob.pos_q, grid)
    nd = np.zeros(nx * ny * nz)
    np.add.at(nd, nodes[donors], 1.0)
    n_elec = float(len(donors))
    U = np.array(U0, dtype=np.float64).reshape(nz, ny, nx).copy()
    res_hist, iterates, rhos, outs, efs = [], [], [], [], []
    converged = False
    for it in range(max_iter):
        o = loop_body(H0, n_o, nodes, nd, U, grid, sigma_mid, n_elec, kT, h, eps_r, Ef_fixed, cg_tol)
        Uout = o["U_out"]
        res = float(np.abs(Uout - U).max())
        res_hist.append(res)
        efs.append(o["Ef"])
        if keep_iterates:
            iterates.append(U.copy())
            rhos.append(o["rho"])
            outs.append(Uout)
        if res < tol:
            converged = True
            break
        U = U + alpha * (Uout - U)
    return dict(U=U, iterations=len(res_hist), residuals=res_hist, iterates=iterates, rhos=rhos,
                outputs=outs, Ef=efs, converged=converged)
