"""Pins for the oracle's block Lanczos: the full Krylov space reproduces the
dense spectrum with every multiplicity (also multiplicities above the block
size, through deflation), the block three-term recurrence holds, Kramers
pairs of a spin-orbit Hamiltonian appear twice, and an exactly invariant
start block is reproduced in one step."""
import numpy as np
import pytest

import workloads as W
from oracle import block_lanczos as BL
from oracle import lanczos as L
from oracle import tb as T


def _dense(p):
    H = T.hamiltonian(p).toarray()
    return H, np.linalg.eigvalsh(H)


def _groups(ev, tol):
    g = [[ev[0]]]
    for e in ev[1:]:
        if e - g[-1][-1] < tol:
            g[-1].append(e)
        else:
            g.append([e])
    return [(float(np.mean(x)), len(x)) for x in g]


@pytest.mark.parametrize("kw,b", [
    (dict(model=W.MODEL_SP3S, strain=True, potential=0.4), 8),          # no degeneracy
    (dict(model=W.MODEL_SP3S), 16),                                        # cubic: multiplicity 20 > b
    (dict(model=W.MODEL_SP3S, spin=1, strain=True, periodic=(0, 0, 0), passivation=30.0), 8),   # Kramers
])
def test_full_krylov_is_the_dense_spectrum(kw, b):
    """m b = n: the Ritz values are every eigenvalue with its multiplicity
    (to 1e-9 eV), and their sum is Tr H."""
    p = W.problem_periodic_cube(2, seed=2, **kw)
    H, ev = _dense(p)
    assert p.dim % b == 0
    rng = np.random.default_rng(0)
    X0 = rng.uniform(-1, 1, (p.dim, b))
    if p.is_complex:
        X0 = X0 + 1j * rng.uniform(-1, 1, (p.dim, b))
    r = BL.block_lanczos(lambda X: H @ X, X0, p.dim // b)
    th = np.linalg.eigvalsh(r["T"])
    assert np.abs(th - ev).max() < 1e-9
    assert abs(th.sum() - np.trace(H).real) < 1e-9 * np.abs(ev).max() * p.dim
    if kw.get("model") == W.MODEL_SP3S and not kw.get("spin") and not kw.get("strain"):
        assert max(c for _, c in _groups(ev, 1e-8)) > b          # deflation was needed


@pytest.mark.parametrize("spin", [0, 1])
def test_block_recurrence_and_orthonormality(spin):
    """H [Q_1..Q_m] = [Q_1..Q_m] T_m + Q_{m+1} B_{m+1} E_m^H and the basis is
    orthonormal; T_m is Hermitian with upper-triangular sub-diagonal blocks."""
    p = W.problem_periodic_cube(2, seed=4, model=W.MODEL_SP3D5S, spin=spin, strain=True,
                                kfrac=(0.1, 0.0, -0.2) if spin else None)
    H = T.hamiltonian(p)
    b, m = 8, 12
    rng = np.random.default_rng(1)
    X0 = rng.uniform(-1, 1, (p.dim, b)) + (1j * rng.uniform(-1, 1, (p.dim, b)) if p.is_complex else 0)
    r = BL.block_lanczos(lambda X: H @ X, X0, m)
    Q = r["Q"]
    Qm = Q[:, :m * b]
    E = Q[:, m * b:] @ r["B"][m]
    lhs = H @ Qm
    rhs = Qm @ r["T"]
    rhs[:, (m - 1) * b:] += E
    hn = abs(H).max() * 50
    assert np.abs(lhs - rhs).max() < 1e-12 * hn
    assert np.abs(Q.conj().T @ Q - np.eye((m + 1) * b)).max() < 1e-12
    assert np.abs(r["T"] - r["T"].conj().T).max() == 0
    for Bj in r["B"][1:]:
        assert np.abs(np.tril(Bj, -1)).max() == 0


def test_short_recurrence_without_reorthogonalisation():
    """A few steps without reorthogonalisation: the three-term block
    recurrence alone keeps the basis orthonormal (to 1e-10 this early) and
    H Q_m = Q_m T_m + Q_{m+1} B_{m+1} E_m^H holds; the coupling term
    Q_{j-1} B_j^H is what makes it hold."""
    p = W.problem_periodic_cube(2, seed=8, model=W.MODEL_SP3D5S, strain=True, potential=0.2)
    H = T.hamiltonian(p)
    b, m = 8, 4
    X0 = np.random.default_rng(5).uniform(-1, 1, (p.dim, b))
    r = BL.block_lanczos(lambda X: H @ X, X0, m, reorth=False)
    Q = r["Q"]
    Qm = Q[:, :m * b]
    rhs = Qm @ r["T"]
    rhs[:, (m - 1) * b:] += Q[:, m * b:] @ r["B"][m]
    assert np.abs(H @ Qm - rhs).max() < 1e-10 * abs(H).max()
    assert np.abs(Q.T @ Q - np.eye((m + 1) * b)).max() < 1e-10


def test_kramers_pairs_appear_twice():
    """Spin-orbit, strained hard-wall cube: every eigenvalue is a Kramers
    pair.  Block Lanczos (b = 4) reports each converged value twice and they
    are eigenvalues of the dense H; scalar Lanczos sees each pair once."""
    p = W.problem_periodic_cube(2, seed=2, model=W.MODEL_SP3S, spin=1, strain=True, periodic=(0, 0, 0),
                                passivation=30.0)
    H, ev = _dense(p)
    rng = np.random.default_rng(3)
    X0 = rng.uniform(-1, 1, (p.dim, 4)) + 1j * rng.uniform(-1, 1, (p.dim, 4))
    r = BL.block_lanczos_eigs(lambda X: H @ X, X0, 160, 0.5, 12, res_tol=1e-8)
    th = np.sort(r["theta"])
    assert th.size == 12
    assert np.abs(th[0::2] - th[1::2]).max() < 1e-8
    for t in th:
        assert np.abs(ev - t).min() < 1e-9
    rs = L.lanczos_eigs(lambda v: H @ v, p.v0, 640, 0.5, 6)
    assert (np.asarray(rs["copies"]) >= 1).all()
    # distinct values nearest sigma: the block result's pairs, one each in the scalar result
    assert np.abs(np.sort(rs["theta"]) - th[0::2]).max() < 1e-8


def test_invariant_start_block_in_one_step():
    """A start block of exact eigenvectors spans an invariant subspace: one
    step gives A_1 = Q_1^H H Q_1 with exactly those eigenvalues, W = 0
    deflates, and the Ritz values are the chosen eigenvalues."""
    p = W.problem_periodic_cube(1, seed=6, model=W.MODEL_SP3D5S, strain=True, potential=0.3)
    H = T.hamiltonian(p).toarray()
    ev, V = np.linalg.eigh(H)
    pick = [3, 7, 11, 19, 30, 41]
    rng = np.random.default_rng(2)
    X0 = V[:, pick] @ rng.standard_normal((6, 6))
    r = BL.block_lanczos(lambda X: H @ X, X0, 1)
    assert np.abs(np.linalg.eigvalsh(r["T"]) - ev[pick]).max() < 1e-12
    assert np.abs(r["B"][1]).max() < 1e-10
    assert (np.diag(r["B"][1]) == 0).all()           # every column deflated
    # the deflated next block is still orthonormal and orthogonal to Q_1
    Q = r["Q"]
    assert np.abs(Q.T @ Q - np.eye(12)).max() < 1e-12


def test_deflation_vector_generator():
    """SplitMix64 replacement values: uniform on [-1, 1) (mean 0, variance
    1/3 within sampling error), distinct counters give distinct values, and
    the generator is a bijection on the sample (no repeated outputs)."""
    u = BL.deflation_vector(3, 5, 16, 200_000, False)
    assert u.min() >= -1 and u.max() < 1
    assert abs(u.mean()) < 4 * np.sqrt(1 / 3 / u.size)
    assert abs(u.var() - 1 / 3) < 0.01
    s = BL.splitmix64(np.arange(100_000, dtype=np.uint64))
    assert np.unique(s).size == s.size
    assert not np.array_equal(BL.deflation_vector(1, 0, 16, 64, False), BL.deflation_vector(1, 1, 16, 64, False))


def test_splitmix64_published_outputs():
    """The counter form mix(x + golden gamma) reproduces the first three
    outputs of the stateful SplitMix64 generator seeded with 0 (Steele, Lea
    and Flood, OOPSLA 2014; the values quoted with the reference C code of the
    xoshiro family): output k is mix(k * gamma)."""
    g = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        x = np.array([0, g, g * np.uint64(2)], dtype=np.uint64)
        s = BL.splitmix64(x)
    assert [int(v) for v in s] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
