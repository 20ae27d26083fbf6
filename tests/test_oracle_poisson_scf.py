"""Pins for the oracle's Poisson solver, Fermi-level search and SCF pieces:
an independent spectral solve of the same discrete equations, exact discrete
eigenfunctions, the lattice Green's function of a point charge, neutrality
and zero-temperature limits."""
import numpy as np
import pytest

from oracle import poisson as P
from oracle import scf as S


def test_constants():
    assert P.EPS0_E_PER_V_NM == pytest.approx(0.0552634936, rel=1e-9)
    # e^2 / (4 pi eps0 eps_r) for eps_r = 11.7
    assert P.COULOMB_EV_NM / 11.7 == pytest.approx(0.123074, rel=1e-5)


@pytest.mark.parametrize("shape", [(6, 4, 4), (12, 8, 6), (9, 5, 7)])
def test_cg_matches_spectral(shape):
    rng = np.random.default_rng(sum(shape))
    b = rng.standard_normal(shape)
    h = 0.135775
    x, it, rr = P.cg(b, h, rel_tol=1e-13)
    xs = P.spectral_solve(b, h)
    assert rr <= 1e-13
    assert np.abs(x - xs).max() <= 1e-10 * np.abs(xs).max()
    assert np.abs(P.neg_laplacian(xs, h) - b).max() <= 1e-9 * np.abs(b).max()


def test_discrete_eigenfunction():
    nz, ny, nx = 10, 6, 8
    h = 0.2
    z = np.arange(nz)[:, None, None]
    y = np.arange(ny)[None, :, None]
    x = np.arange(nx)[None, None, :]
    kz, ky, kx = 3, 1, 2
    f = np.sin(np.pi * kz * (z + 1) / (nz + 1)) * np.cos(2 * np.pi * ky * y / ny) * np.cos(2 * np.pi * kx * x / nx)
    lam = ((2 - 2 * np.cos(np.pi * kz / (nz + 1))) + (2 - 2 * np.cos(2 * np.pi * ky / ny))
           + (2 - 2 * np.cos(2 * np.pi * kx / nx))) / h ** 2
    assert np.abs(P.neg_laplacian(f, h) - lam * f).max() < 1e-10 * lam


def test_point_charge_lattice_green_function():
    """A unit charge on a large grid: the potential at the charge node tends
    to G0 e/(eps0 eps_r h) with the simple-cubic lattice Green's function
    G0 = 0.2527310098; at distance r it tends to e/(4 pi eps0 eps_r r)."""
    n = 96
    h = 0.135775
    eps_r = 11.7
    rho = np.zeros((n, n, n))
    c = n // 2
    rho[c, c, c] = 1.0 / h ** 3
    phi = P.spectral_solve(P.rhs(rho, eps_r), h)
    g0 = phi[c, c, c] * P.EPS0_E_PER_V_NM * eps_r * h
    # finite box (grounded z plates, periodic images in x, y) lowers it by O(h/L)
    assert g0 == pytest.approx(0.2527310098, rel=0.02)
    r = 6
    coul = P.COULOMB_EV_NM / eps_r / (r * h)
    assert phi[c, c, c + r] == pytest.approx(coul, rel=0.05)


def test_fermi_neutrality_and_limits():
    rng = np.random.default_rng(0)
    E = np.sort(rng.uniform(-1, 1, 40))
    kT = S.KB_EV * 4.0
    for ne in (1.0, 7.0, 16.0, 33.0):
        Ef = S.fermi_level(E, ne, kT)
        assert 2 * S.occupation(E, Ef, kT).sum() == pytest.approx(ne, abs=1e-10)
    # zero temperature: integer filling of the lowest levels
    Ef = S.fermi_level(E, 16.0, 0.0)
    occ = S.occupation(E, Ef, 0.0)
    assert np.array_equal(occ[:8], np.ones(8)) and occ[8:].sum() == 0
    # a given Fermi level (fixed-E_F mode) at 4 K is a step away from E_F
    occ = S.occupation(E, 0.0, kT)
    assert np.allclose(occ, (E < 0).astype(float), atol=1e-12)


def test_density_counts_electrons():
    rng = np.random.default_rng(1)
    n_atoms, n_o = 6, 3
    Q, _ = np.linalg.qr(rng.standard_normal((n_atoms * n_o, n_atoms * n_o)))
    E = np.sort(rng.uniform(0, 1, n_atoms * n_o))
    w = S.atom_weights(Q, n_o)
    assert np.allclose(w.sum(axis=1), 1.0)
    n, Ef, cb = S.electron_density(E, w, np.zeros(n_atoms), -1.0, 5.0, S.KB_EV * 4)
    assert n.sum() == pytest.approx(5.0, abs=1e-10)
