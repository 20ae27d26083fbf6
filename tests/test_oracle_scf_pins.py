"""Pins for the parts of the oracle that the trace identities cannot see:
the direction of the dangling-bond hybrid (Sec. I hard-wall structures), the
sign of the electron potential energy (Sec. III-A item 3: donors attract
electrons), and the body of the self-consistent loop (Sec. III-A items 2-3:
charge from the filled states, Poisson, mixing).

Every expected value here is built from something other than the oracle's
own formula: lattice positions instead of the slot-direction table, the
maximum principle of the discrete Laplacian, the electrostatics of a charged
sheet between grounded plates, and dense eigenpairs of H(U) assembled through
the per-atom on-site route instead of the loop's diagonal shift.
"""
import numpy as np
import pytest

import workloads as W
from oracle import poisson as P
from oracle import scf as S
from oracle import tb as T


def _lattice_site(p):
    """True where integer a/4 coordinates p lie on the infinite diamond lattice:
    all even with x+y+z = 0 (mod 4), or all odd with x+y+z = 3 (mod 4)."""
    p = np.asarray(p)
    s = p.sum(axis=-1) % 4
    even = (p % 2 == 0).all(axis=-1)
    odd = (p % 2 == 1).all(axis=-1)
    return (even & (s == 0)) | (odd & (s == 3))


def _missing_neighbour_displacements(pos, box, periodic):
    """For each atom, the displacements d in {+-1}^3 to lattice sites that are
    nearest neighbours of the infinite crystal but lie outside a hard wall."""
    out = []
    for q in pos:
        miss = []
        for d in np.array(np.meshgrid([-1, 1], [-1, 1], [-1, 1], indexing="ij")).reshape(3, -1).T:
            t = q + d
            if not _lattice_site(t):
                continue
            inside = all(periodic[ax] or 0 <= t[ax] < box[ax] for ax in range(3))
            if not inside:
                miss.append(d)
        out.append(miss)
    return out


@pytest.mark.parametrize("spin", [0, 1])
@pytest.mark.parametrize("periodic", [(0, 0, 0), (1, 1, 0)])
def test_passivation_hybrid_points_at_missing_neighbour(spin, periodic):
    """D_passivated - D_bare = E_pass sum_missing |h><h| with h = (s + d.p)/2,
    d the displacement from the atom to its missing neighbour, found from the
    positions alone; checked on both sublattices (and both spins)."""
    e_pass = 30.0
    kw = dict(model=W.MODEL_SP3D5S, spin=spin, periodic=periodic, nxyz=(2, 2, 2))
    p0 = W.problem_periodic_cube(0, seed=5, **kw)
    p1 = W.problem_periodic_cube(0, seed=5, passivation=e_pass, **kw)
    D = T.build_blocks(p1)["onsite"] - T.build_blocks(p0)["onsite"]
    miss = _missing_neighbour_displacements(p0.pos_q, p0.box_q, p0.periodic)
    nb = 10
    sub = (p0.pos_q.sum(axis=1) % 4 == 3)
    seen = set()
    for i, dl in enumerate(miss):
        want = np.zeros((nb, nb))
        for d in dl:
            h = np.zeros(nb)
            h[0] = 0.5
            h[1:4] = 0.5 * d          # p_x, p_y, p_z follow s in the orbital order
            want += e_pass * np.outer(h, h)
        if spin:
            want = np.kron(np.eye(2), want)
        assert np.abs(D[i] - want).max() < 1e-12, (i, p0.pos_q[i], dl)
        if dl:
            seen.add(bool(sub[i]))
    assert seen == {False, True}, "both sublattices must carry dangling bonds"


def test_hybrid_sign_matters():
    """The check above would see a reversed hybrid: (s - d.p)/2 differs from
    (s + d.p)/2 in every s-p element of the projector."""
    d = np.array([1, -1, -1])
    hp = np.r_[0.5, 0.5 * d]
    hm = np.r_[0.5, -0.5 * d]
    assert np.abs(np.outer(hp, hp) - np.outer(hm, hm)).max() == pytest.approx(0.5)


def test_positive_charge_lowers_electron_energy():
    """A single +e ion: phi > 0 everywhere inside grounded plates (maximum
    principle of the discrete Laplacian with a non-negative source), so the
    electron potential energy U = -phi is negative everywhere and deepest at
    the ion's node."""
    nz, ny, nx = 12, 8, 8
    h = W.H_GRID_NM
    rho = np.zeros((nz, ny, nx))
    c = (5, 3, 4)
    rho[c] = 1.0 / h ** 3
    U, it, rr = P.potential_energy(rho, h, 11.7, rel_tol=1e-13)
    assert rr <= 1e-13
    assert (U < 0).all()
    assert np.unravel_index(np.argmin(U), U.shape) == c
    # it is the same solution as the independent spectral solve, with the sign flipped
    assert np.abs(U + P.spectral_solve(P.rhs(rho, 11.7), h)).max() < 1e-9 * np.abs(U).max()


def _slab(nz=4, nxy=1, n_donors=1, plane=None, seed=0):
    """A small delta-doped slab in the C5 geometry (periodic x, y, hard-wall z,
    +30 eV passivation, sp3d5s* with the gap-accepted parameters), donors on
    the (001) plane z = plane (a/4 units; default the mid plane)."""
    p = W.c5_slab(seed, nx=nxy, ny=nxy, nz=nz, n_donors=n_donors)
    if plane is not None:
        rng = np.random.default_rng(seed + 17)
        p.extra["donor_atoms"] = W.draw_donor_sites(rng, p.pos_q, plane_qz=plane, n_donors=n_donors)
    return p


def test_donor_plane_is_the_potential_minimum_after_one_step():
    """One step from the zero start with the donor plane off centre: the
    donors' sheet of positive charge between grounded plates gives a
    potential-energy profile with its minimum at the sheet, while the
    electrons of the flat start spread over the slab.  So the new potential
    is lower on the donor plane than on its mirror plane; a reversed sign of
    rho or of U = -phi reverses the inequality."""
    nz = 4
    zp = 4                      # a quarter of the slab's 16 planes
    p = _slab(nz=nz, nxy=1, n_donors=2, plane=zp)
    grid = p.extra["grid"]
    gap = p.extra["gap"]
    r = S.scf(p, p.extra["donor_atoms"], grid, np.zeros(grid[::-1]), gap["mid"], alpha=0.5, tol=0.0,
              max_iter=1)
    U = r["U"]
    zm = grid[2] - 1 - zp
    on_plane = p.pos_q[:, 2] == zp
    on_mirror = p.pos_q[:, 2] == zm
    q = p.pos_q
    u_plane = U[q[on_plane, 2], q[on_plane, 1], q[on_plane, 0]].mean()
    u_mirror = U[q[on_mirror, 2], q[on_mirror, 1], q[on_mirror, 0]].mean()
    assert u_plane < u_mirror - 1e-3, (u_plane, u_mirror)
    # and the electrons of the next step gather towards the donor plane
    r2 = S.scf(p, p.extra["donor_atoms"], grid, U, gap["mid"], alpha=0.5, tol=0.0, max_iter=1)
    rho_e = -(r2["rhos"][0] * W.H_GRID_NM ** 3)      # electrons minus donors
    nd = W.donor_map(q, p.extra["donor_atoms"], grid)
    ne = rho_e + nd                                     # electrons per node
    z = np.arange(grid[2])[:, None, None]
    zc = (ne * z).sum() / ne.sum()
    assert abs(zc - zp) < abs(zc - zm), (zc, zp, zm)


@pytest.mark.parametrize("shift", [0.0, -3.0])
def test_one_occupied_state_charge_density(shift):
    """Fixed Fermi level between the two lowest conduction-band-like states at
    T = 0: exactly one state holds two electrons, so rho at the node of atom i
    is e (N_D(i) - 2 sum_alpha |psi_1(i, alpha)|^2) / h^3 and zero on empty
    nodes.  The eigenpair comes from a dense solve of H(U) built with U on the
    per-atom on-site blocks; node (x, y, z) has index (z ny + y) nx + x.
    A uniform shift of U by 3 eV moves this small slab's conduction band
    below the gap centre; a state is still conduction-band-like by its energy
    less its mean potential, so the same state is the one filled."""
    p = _slab(nz=3, nxy=1, n_donors=1, seed=2)
    grid = p.extra["grid"]
    nx, ny, nz = grid
    gap = p.extra["gap"]
    rng = np.random.default_rng(9)
    U0 = shift + rng.uniform(-0.05, 0.05, size=(nz, ny, nx))       # breaks every degeneracy
    q = p.pos_q
    Ua = U0[q[:, 2], q[:, 1], q[:, 0]]
    pu = W.problem_periodic_cube(0, seed=0, model=W.MODEL_SP3D5S, spin=0, periodic=(1, 1, 0),
                                 nxyz=(1, 1, 3), passivation=30.0, param_seed=gap["seed"])
    pu.onsite_pot = Ua
    Hm = T.hamiltonian(pu).toarray()
    E, psi = np.linalg.eigh(Hm)
    n_o = 10
    w = (psi ** 2).T.reshape(len(E), -1, n_o).sum(axis=2)
    cb = np.flatnonzero(E - w @ Ua > gap["mid"])
    e1, e2 = E[cb[0]], E[cb[1]]
    if shift:
        assert e1 < gap["mid"]        # below the gap centre, counted only through E - <U>
    assert e2 - e1 > 1e-6
    ef = 0.5 * (e1 + e2)
    r = S.scf(p, p.extra["donor_atoms"], grid, U0, gap["mid"], alpha=0.1, tol=0.0, max_iter=1, T_K=0.0,
              Ef_fixed=ef)
    h = W.H_GRID_NM
    want = np.zeros(nx * ny * nz)
    node = (q[:, 2] * ny + q[:, 1]) * nx + q[:, 0]
    d = p.extra["donor_atoms"]
    want[node[d]] += 1.0
    want[node] -= 2.0 * w[cb[0]]
    want = want.reshape(nz, ny, nx) / h ** 3
    assert np.abs(r["rhos"][0] - want).max() <= 1e-10 * np.abs(want).max()
    # one state, two electrons, one donor: net charge -1 e
    assert (r["rhos"][0].sum() * h ** 3) == pytest.approx(1.0 - 2.0, abs=1e-10)


def test_neutrality_and_mixing_every_step():
    """With the Fermi level from neutrality the total charge is zero at every
    step, and each step's input is the previous input moved by alpha towards
    that step's output."""
    p = _slab(nz=3, nxy=1, n_donors=1, seed=4)
    grid = p.extra["grid"]
    alpha = 0.3
    r = S.scf(p, p.extra["donor_atoms"], grid, np.zeros(grid[::-1]), p.extra["gap"]["mid"], alpha=alpha,
              tol=0.0, max_iter=4)
    h3 = W.H_GRID_NM ** 3
    for t in range(4):
        assert abs(r["rhos"][t].sum() * h3) < 1e-10
        # the residual is the max-norm distance of input and output
        assert r["residuals"][t] == pytest.approx(np.abs(r["outputs"][t] - r["iterates"][t]).max(), rel=1e-14)
    for t in range(3):
        step = r["iterates"][t + 1] - r["iterates"][t]
        assert np.abs(step - alpha * (r["outputs"][t] - r["iterates"][t])).max() < 1e-12


def test_converged_potential_is_a_fixed_point():
    """At the oracle's converged U, the output potential computed here from a
    dense eigen-solve, a Fermi level by neutrality and the spectral Poisson
    solve (not the loop's CG) equals U to the loop tolerance."""
    p = _slab(nz=3, nxy=1, n_donors=1, seed=6)
    grid = p.extra["grid"]
    nx, ny, nz = grid
    gap = p.extra["gap"]
    tol = 1e-7
    r = S.scf(p, p.extra["donor_atoms"], grid, np.zeros((nz, ny, nx)), gap["mid"], alpha=0.3, tol=tol,
              max_iter=400, keep_iterates=False)
    assert r["converged"]
    U = r["U"]
    q = p.pos_q
    Ua = U[q[:, 2], q[:, 1], q[:, 0]]
    pu = W.problem_periodic_cube(0, seed=0, model=W.MODEL_SP3D5S, spin=0, periodic=(1, 1, 0),
                                 nxyz=(1, 1, 3), passivation=30.0, param_seed=gap["seed"])
    pu.onsite_pot = Ua
    E, psi = np.linalg.eigh(T.hamiltonian(pu).toarray())
    w = (psi ** 2).T.reshape(len(E), -1, 10).sum(axis=2)
    cb = E - w @ Ua > gap["mid"]
    kT = S.KB_EV * 4.0
    ef = S.fermi_level(E[cb], 1.0, kT)
    f = S.occupation(E[cb], ef, kT)
    n_atom = 2.0 * (f[:, None] * w[cb]).sum(axis=0)
    rho = np.zeros((nz, ny, nx))
    d = p.extra["donor_atoms"]
    rho[q[d, 2], q[d, 1], q[d, 0]] += 1.0
    np.subtract.at(rho, (q[:, 2], q[:, 1], q[:, 0]), n_atom)
    h = W.H_GRID_NM
    U_out = -P.spectral_solve(P.rhs(rho / h ** 3, 11.7), h)
    assert np.abs(U_out - U).max() < 2 * tol
