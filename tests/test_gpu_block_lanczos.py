"""GPU parity of block Lanczos (and of its projected-matrix eigensolver)
against dense LAPACK spectra and the oracle's block Lanczos.

Bars: the dense eigensolver's eigenpairs nearest the target to 1e-10 |A|
(values, residuals, orthonormality); block Lanczos eigenvalues (FP64
Rayleigh quotients of converged pairs, residual <= 1e-4 eV) within 1e-6 eV of
the dense FP64 spectrum, with every multiplicity counted.
"""
import numpy as np
import pytest

import paper_1003_4570_amd as tbh
import workloads as W
from oracle import block_lanczos as BL
from oracle import tb as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return tbh.Context(0)


def _nearest(ev, sigma, k):
    """The k values nearest sigma (ties: lower value), ascending."""
    idx = np.lexsort((ev, np.abs(ev - sigma)))[:k]
    return np.sort(ev[idx])


@pytest.mark.parametrize("n,nc,kind", [(37, 8, "random"), (64, 64, "random"), (48, 20, "clustered"),
                                       (256, 40, "random"), (700, 64, "clustered"), (1024, 64, "clustered")])
def test_projected_eigensolver_matches_lapack(ctx, n, nc, kind):
    """n <= 64 takes the LDS kernels (one-wavefront reduction, interleaved
    inverse iteration), as in the filtered solver's Rayleigh-Ritz (n = nc =
    64); larger n the global-memory ones."""
    print(f"dense eig n={n} nc={nc} kind={kind}", flush=True)
    rng = np.random.default_rng(n)
    if kind == "random":
        M = rng.standard_normal((n, n))
        A = 0.5 * (M + M.T)
    else:
        # repeated eigenvalues (multiplicities 12 and 5) around the target
        lam = rng.uniform(-10, 10, n)
        lam[:12] = 0.3
        lam[12:17] = 0.31
        Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
        A = (Qm * lam) @ Qm.T
        A = 0.5 * (A + A.T)
    sigma = 0.3
    th, V = tbh.symm_eig_near(ctx, A, sigma, nc)
    ev = np.linalg.eigvalsh(A)
    an = np.abs(ev).max()
    assert np.abs(th - _nearest(ev, sigma, nc)).max() <= 1e-10 * an
    R = A @ V.T - V.T * th[None, :]
    assert np.abs(R).max() <= 1e-10 * an
    assert np.abs(V @ V.T - np.eye(nc)).max() <= 1e-10


def _ham(ctx, p):
    return tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec="f32", keep_f64=True, multi_vector=True))


def test_full_krylov_with_multiplicity_above_block(ctx):
    """Cubic sp3s* 2^3 cell (320 states, one eigenvalue 20-fold): 20 steps of
    block size 16 span the whole space through deflation; the 16 pairs nearest
    1 eV, each copy counted, equal the dense spectrum's."""
    p = W.problem_periodic_cube(2, seed=2, model=W.MODEL_SP3S)
    h = _ham(ctx, p)
    ev = np.linalg.eigvalsh(T.hamiltonian(p).toarray())
    r = tbh.block_lanczos_eigs(h, 1.0, 16, 16, 20)
    print("report", r["report"], flush=True)
    assert r["report"]["n_found"] == 16
    assert np.abs(np.sort(r["refined"]) - _nearest(ev, 1.0, 16)).max() < 1e-6
    assert r["report"]["deflated"] > 0


def test_c1_multiplicities_with_restarts(ctx):
    """C1 (512-atom periodic Si, sp3s*, degeneracies up to 44-fold): the 64
    pairs nearest 1 eV by restarted block Lanczos (b = 64, Krylov space of
    (H - 1 eV)^2, where they are the smallest eigenvalues) equal the dense
    spectrum's 64 nearest with multiplicity, to 1e-6 eV."""
    p = W.c1_lanczos_fp64(0)
    h = _ham(ctx, p)
    ev = np.linalg.eigvalsh(T.hamiltonian(p).toarray())
    r = tbh.block_lanczos_eigs(h, p.sigma, 64, 64, 32, cycles=12, fold=True)
    print("report", r["report"], flush=True)
    assert r["report"]["n_found"] == 64
    assert np.abs(np.sort(r["refined"]) - _nearest(ev, p.sigma, 64)).max() < 1e-6


def test_against_oracle_block_lanczos(ctx):
    """Strained alloy 2^3 cell with a random potential (no degeneracy), the
    same start block on both sides: every pair the oracle's FP64 block
    Lanczos converges among the 8 nearest 1 eV is converged on the GPU with
    the same eigenvalue to 1e-6 eV, and each GPU value is a dense eigenvalue."""
    import torch
    p = W.problem_periodic_cube(2, seed=4, model=W.MODEL_SP3D5S, strain=True, potential=0.3, n_species=2,
                                alloy_frac=0.4)
    H = T.hamiltonian(p)
    ev = np.linalg.eigvalsh(H.toarray())
    b, m = 32, 12
    X0 = np.random.default_rng(7).uniform(-1, 1, (p.dim, b))
    ro = BL.block_lanczos_eigs(lambda X: H @ X, X0, m, 1.0, 8)
    h = _ham(ctx, p)
    x0 = torch.from_numpy(np.ascontiguousarray(X0.T)).cuda()
    r = tbh.block_lanczos_eigs(h, 1.0, 8, b, m, x0=x0)
    print("oracle", ro["theta"], "gpu", r["refined"], flush=True)
    for e in r["refined"]:
        assert np.abs(ev - e).min() < 1e-6
    for e in ro["theta"]:
        assert np.abs(r["refined"] - e).min() < 1e-6


def test_warm_start_of_eigenvectors(ctx):
    """A start block of the 16 exact eigenvectors nearest the target: one
    block step reproduces them (FP32 rounding of the block only), and the
    returned vectors are unit eigenvectors with FP64 residuals <= 1e-4 eV."""
    import torch
    p = W.problem_periodic_cube(2, seed=6, model=W.MODEL_SP3D5S, strain=True, potential=0.3)
    Hd = T.hamiltonian(p).toarray()
    ev, V = np.linalg.eigh(Hd)
    idx = np.sort(np.lexsort((ev, np.abs(ev - 0.5)))[:16])
    h = _ham(ctx, p)
    x0 = torch.from_numpy(np.ascontiguousarray(V[:, idx].T)).cuda()
    r = tbh.block_lanczos_eigs(h, 0.5, 16, 16, 1, x0=x0, want_vectors=True)
    assert r["report"]["n_found"] == 16
    assert np.abs(r["refined"] - ev[idx]).max() < 1e-6
    Y = r["vectors"].cpu().numpy()
    assert np.abs(np.linalg.norm(Y, axis=1) - 1).max() < 1e-12
    assert np.abs(Hd @ Y.T - Y.T * r["refined"][None, :]).max() < 1e-4
