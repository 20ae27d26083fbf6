"""Pins for the CPU oracle's Lanczos eigensolver: dense eigendecomposition,
trace of the full tridiagonal, orthonormality of the basis and the
three-term recurrence."""
import numpy as np
import pytest

import workloads as W
from oracle import lanczos as L
from oracle import tb as T


def _broken(n=1, spin=0, seed=5):
    # symmetry broken by random strain and potential so eigenvalues are simple
    return W.problem_periodic_cube(n, seed=seed, model=W.MODEL_SP3S, spin=spin,
                                   strain=True, potential=0.5, kfrac=(0.1, 0.2, 0.3) if spin else None)


@pytest.mark.parametrize("spin", [0, 1])
def test_full_krylov_equals_dense(spin):
    p = _broken(1, spin)
    H = T.hamiltonian(p)
    dim = H.shape[0]
    a, b, V = L.lanczos(lambda x: H @ x, p.v0, dim)
    assert len(a) == dim
    th, _ = L.tridiag_eig(a, b)
    ev = np.linalg.eigvalsh(H.toarray())
    assert np.abs(np.sort(th) - ev).max() < 1e-9
    assert np.sum(th) == pytest.approx(np.trace(H.toarray()).real, abs=1e-9)


def test_basis_orthonormal_and_recurrence():
    p = _broken(2)
    H = T.hamiltonian(p)
    m = 120
    a, b, V = L.lanczos(lambda x: H @ x, p.v0, m)
    G = V @ V.conj().T
    assert np.abs(G - np.eye(m)).max() < 1e-13
    # H V^T = V^T T + beta_m v_{m+1} e_m^T: check the first m-1 columns
    Tm = np.diag(a) + np.diag(b[:-1], 1) + np.diag(b[:-1], -1)
    R = (H @ V.T) - V.T @ Tm
    assert np.abs(R[:, :-1]).max() < 1e-11


@pytest.mark.parametrize("seed", [0, 11])
def test_c1_nearest_distinct_match_dense(seed):
    p = W.c1_lanczos_fp64(0)
    rng = np.random.default_rng(seed + 100)
    v0 = rng.uniform(-1, 1, p.dim)
    H = T.hamiltonian(p)
    r = L.lanczos_eigs(lambda x: H @ x, v0, p.m, p.sigma, p.k)
    ev = np.linalg.eigvalsh(H.toarray())
    # distinct dense eigenvalues (multiplicities from the cubic symmetry)
    u = [ev[0]]
    for e in ev[1:]:
        if e - u[-1] > 1e-8:
            u.append(e)
    u = np.array(u)
    want = np.sort(u[np.argsort(np.abs(u - p.sigma), kind="stable")[:p.k]])
    assert len(r["theta"]) == p.k
    assert np.abs(r["theta"] - want).max() < 1e-6
    assert np.abs(r["refined"] - want).max() < 1e-9
    assert (r["res"] <= 1e-4).all()


def test_c1_without_reorth_ghosts_merge_to_dense_values():
    """Without reorthogonalisation converged values reappear as ghost
    copies; after merging, the 8 distinct values nearest sigma still equal
    the dense spectrum's (each with more than one copy at 600 steps)."""
    p = W.c1_lanczos_fp64(0)
    H = T.hamiltonian(p)
    r = L.lanczos_eigs(lambda x: H @ x, p.v0, 600, p.sigma, p.k, reorth=False)
    ev = np.linalg.eigvalsh(H.toarray())
    u = [ev[0]]
    for e in ev[1:]:
        if e - u[-1] > 1e-8:
            u.append(e)
    u = np.array(u)
    want = np.sort(u[np.argsort(np.abs(u - p.sigma), kind="stable")[:p.k]])
    assert len(r["theta"]) == p.k
    assert np.abs(r["refined"] - want).max() < 1e-9
    assert (np.asarray(r["copies"]) >= 2).any()


def test_selection_rule():
    th = np.array([0.9, 1.0000001, 1.0000004, 1.3, 0.2, 5.0])
    res = np.array([1e-9, 1e-6, 1e-8, 1e-3, 1e-10, 1e-12])
    sel = L.select_converged(th, res, th + 1e-12, sigma=1.0, k=3)
    # 1.0000001 and 1.0000004 merge (copy count 2, representative = smaller residual)
    assert np.allclose(sel["theta"], [0.2, 0.9, 1.0000004])
    assert list(sel["copies"]) == [1, 1, 2]
    # unconverged 1.3 is never reported
    sel = L.select_converged(th, res, th, sigma=1.3, k=1)
    assert np.allclose(sel["theta"], [1.0000004])


def test_breakdown_on_eigenvector_start():
    p = _broken(1)
    H = T.hamiltonian(p).toarray()
    w, U = np.linalg.eigh(H)
    a, b, V = L.lanczos(lambda x: H @ x, U[:, 3], 50)
    assert len(a) == 1 and a[0] == pytest.approx(w[3], abs=1e-12)
