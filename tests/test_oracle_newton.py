"""Pins of the Newton-Raphson update's oracle (oracle/newton.py) on the CPU.

* The response chi over ALL eigenstates equals the central finite
  difference of the loop's density rule through dense eigen-solves (300 K,
  neutrality and given Fermi level): this fixes the perturbation formula,
  its factor 2, g_ik, the Fermi-level term and the signs.
* chi conserves charge under neutrality (sum_j (chi v)_j = 0), and is
  symmetric and negative semi-definite, also when truncated to a few states.
* The grid operator equals the oracle's stencil.
* With the exact Jacobian and no Anderson mixing the residual falls
  quadratically near the solution (300 K).
* Anderson mixing of depth >= n solves an n-dimensional affine fixed-point
  problem in at most n + 2 iterations (it is GMRES in disguise there);
  depth 0 is the plain iteration.
* At 4 K with 64 states and Anderson depth 4, the update converges and its
  result is a fixed point of the plain loop body (an independent check of
  the converged potential).
"""
import numpy as np
import pytest

import workloads as W
from oracle import newton as N
from oracle import poisson as P
from oracle import scf as S
from oracle import tb as T


def _setup(nx=1, ny=1, nz=2, n_donors=1, seed=0):
    p = W.c5_slab(seed, nx=nx, ny=ny, nz=nz, n_donors=n_donors)
    grid = p.extra["grid"]
    blk = T.build_blocks(p)
    H0 = T.csr_hamiltonian(blk).toarray()
    nodes = S.node_index(p.pos_q, grid)
    return p, grid, blk["n_o"], H0, nodes


def _density(H0, n_o, nodes, Ua, sigma_mid, n_elec, kT, Ef=None):
    E, psi = np.linalg.eigh(H0 + np.diag(np.repeat(Ua, n_o)))
    wts = S.atom_weights(psi, n_o)
    n, Ef, cb = S.electron_density(E, wts, Ua, sigma_mid, n_elec, kT, Ef)
    return n, Ef, E, psi, cb


@pytest.mark.parametrize("fixed", [False, True])
def test_response_equals_finite_difference(fixed):
    p, grid, n_o, H0, nodes = _setup()
    ge = p.extra["gap"]
    kT = 0.025
    rng = np.random.default_rng(3)
    Ua = rng.uniform(-0.3, 0.0, len(nodes))
    n_elec = 1.0
    n0, Ef, E, psi, cb = _density(H0, n_o, nodes, Ua, ge["mid"], n_elec, kT)
    Ef_in = Ef if fixed else None
    # all states: the counted ones fill by Fermi-Dirac, the rest (valence)
    # stay empty but their mixing with the filled states moves charge
    chi = N.response_matrix(psi, n_o, E, Ef, kT, fixed=fixed, counted=cb)
    v = rng.standard_normal(len(nodes))
    eps = 1e-5
    n_p = _density(H0, n_o, nodes, Ua + eps * v, ge["mid"], n_elec, kT, Ef_in)[0]
    n_m = _density(H0, n_o, nodes, Ua - eps * v, ge["mid"], n_elec, kT, Ef_in)[0]
    fd = (n_p - n_m) / (2 * eps)
    got = chi @ v
    assert np.abs(got - fd).max() <= 1e-6 * np.abs(fd).max()
    assert np.abs(fd).max() > 1e-3          # the perturbation does move charge


def test_response_conserves_charge_symmetric_negative():
    p, grid, n_o, H0, nodes = _setup(2, 2, 2, 1)
    Ua = np.random.default_rng(1).uniform(-0.2, 0.0, len(nodes))
    E, psi = np.linalg.eigh(H0 + np.diag(np.repeat(Ua, n_o)))
    wts = S.atom_weights(psi, n_o)
    cb = E - wts @ Ua > p.extra["gap"]["mid"]
    Ec, Pc = E[cb], psi[:, cb]
    Ef = Ec[0] + 0.004
    for k in (3, 12):
        chi = N.response_matrix(Pc[:, :k], n_o, Ec[:k], Ef, 0.01)
        assert np.abs(chi - chi.T).max() <= 1e-12 * np.abs(chi).max()
        assert np.linalg.eigvalsh(chi).max() <= 1e-10 * np.abs(chi).max()
        assert np.abs(chi.sum(axis=0)).max() <= 1e-10 * np.abs(chi).max()


def test_grid_operator_is_the_stencil():
    grid = (4, 6, 5)
    h = 0.3
    A = N.neg_laplacian_matrix(grid, h)
    x = np.random.default_rng(2).standard_normal(grid[::-1])
    assert np.abs(A @ x.ravel() - P.neg_laplacian(x, h).ravel()).max() < 1e-10


def test_exact_newton_converges_quadratically():
    p, grid, n_o, H0, nodes = _setup(1, 1, 3, 1)
    ge = p.extra["gap"]
    donors = p.extra["donor_atoms"]
    U0 = np.zeros(grid[::-1])
    r = N.scf_newton(p, donors, grid, U0, ge["mid"], tol=1e-11, max_iter=12, T_K=300.0, kT_J=S.KB_EV * 300.0,
                     depth=0, exact=True)
    res = r["residuals"]
    print("residuals", ["%.2e" % x for x in res])
    assert r["converged"]
    # once in the quadratic region each residual is below C r^2 with C ~ 1/eV
    tail = [i for i in range(1, len(res)) if res[i - 1] < 1e-2]
    assert tail
    for i in tail:
        assert res[i] <= 10.0 * res[i - 1] ** 2 + 1e-11


def test_anderson_solves_affine_problem():
    rng = np.random.default_rng(5)
    n = 6
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    M = (Q * rng.uniform(-0.95, 0.95, n)) @ Q.T
    c = rng.standard_normal(n)
    xstar = np.linalg.solve(np.eye(n) - M, c)
    x = np.zeros(n)
    Xs, Fs = [], []
    for it in range(n + 2):
        f = M @ x + c - x
        Xs.append(x.copy())
        Fs.append(f)
        Xs, Fs = Xs[-(n + 1):], Fs[-(n + 1):]
        x = N.anderson(Xs, Fs)
    assert np.abs(x - xstar).max() < 1e-9 * np.abs(xstar).max()
    # depth 0: the plain fixed-point iteration
    x0 = rng.standard_normal(n)
    assert np.allclose(N.anderson([x0], [M @ x0 + c - x0]), M @ x0 + c)


def test_newton_at_4K_reaches_a_fixed_point_of_the_loop():
    p = W.c5_slab(0, nx=2, ny=2, nz=4, n_donors=3)
    grid = p.extra["grid"]
    ge = p.extra["gap"]
    donors = p.extra["donor_atoms"]
    r = N.scf_newton(p, donors, grid, np.zeros(grid[::-1]), ge["mid"], tol=1e-8, max_iter=25)
    print("residuals", ["%.2e" % x for x in r["residuals"]])
    assert r["converged"] and r["iterations"] <= 15
    blk = T.build_blocks(p)
    H0 = T.csr_hamiltonian(blk).toarray()
    nodes = S.node_index(p.pos_q, grid)
    nd = np.zeros(int(np.prod(grid)))
    np.add.at(nd, nodes[donors], 1.0)
    o = S.loop_body(H0, blk["n_o"], nodes, nd, r["U"], grid, ge["mid"], float(len(donors)), S.KB_EV * 4.0,
                    W.H_GRID_NM, 11.7, None, 1e-13)
    assert np.abs(o["U_out"] - r["U"]).max() < 1e-8
