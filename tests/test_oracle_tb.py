"""Pins for the CPU oracle's tight-binding Hamiltonian.

Each test checks the oracle against something other than itself: brute-force
neighbour search, lattice counts, values of the Slater-Koster table at
special directions, the Gamma-point closed form of bulk sp3s*, the L.S
spectrum, trace identities and the folding of bulk bands onto a supercell.
"""
import numpy as np
import pytest

import workloads as W
from oracle import tb as T


def _cube(n, periodic=(1, 1, 1), **kw):
    return W.problem_periodic_cube(n, seed=3, periodic=periodic, **kw)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_atom_count(n):
    assert W.diamond_positions(n, n, n).shape == (8 * n ** 3, 3)
    # 80 cells per edge is the 4-million-atom cube of Sec. II-B (Fig. 3)
    assert 8 * 80 ** 3 == 4_096_000


@pytest.mark.parametrize("n,periodic", [(1, (1, 1, 1)), (2, (1, 1, 1)), (2, (0, 0, 0)),
                                        (2, (1, 1, 0)), (3, (1, 0, 1))])
def test_neighbours_match_brute_force(n, periodic):
    p = _cube(n, periodic)
    nbr, wrap = T.find_neighbours(p.pos_q, p.box_q, p.periodic)
    bf = T.brute_force_neighbours(p.pos_q, p.box_q, p.periodic)
    for i in range(p.n_atoms):
        assert set(int(j) for j in nbr[i] if j >= 0) == bf[i]
        # positions agree with the recorded wrap
        for b in range(4):
            j = nbr[i, b]
            if j < 0:
                continue
            d = T.SLOT_DIRS[b] * (1 if T.sublattice(p.pos_q[i:i + 1])[0] == 0 else -1)
            assert np.array_equal(p.pos_q[j] + wrap[i, b] * np.array(p.box_q), p.pos_q[i] + d)


@pytest.mark.parametrize("n", [1, 2, 4])
def test_periodic_four_distinct_and_reverse_slot(n):
    p = _cube(n)
    nbr, wrap = T.find_neighbours(p.pos_q, p.box_q, p.periodic)
    assert (nbr >= 0).all()
    assert all(len(set(r)) == 4 for r in nbr.tolist())
    for b in range(4):
        assert np.array_equal(nbr[nbr[:, b], b], np.arange(p.n_atoms))
        assert np.array_equal(wrap[nbr[:, b], b], -wrap[:, b])


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_hardwall_dangling_count(n):
    p = _cube(n, (0, 0, 0))
    nbr, _ = T.find_neighbours(p.pos_q, p.box_q, p.periodic)
    assert int((nbr < 0).sum()) == 24 * n * n - 6 * n


def test_sk_table_special_directions():
    """Rotation-built blocks against entries of the Slater-Koster table
    evaluated at (1,1,1)/sqrt3 and (1,0,0)."""
    rng = np.random.default_rng(0)
    V = rng.uniform(-3, 3, 14)
    s3 = np.sqrt(3.0)
    B = T.sk_block(T.MODEL_SP3D5S, V, [1, 1, 1])
    s, px, py, pz, dxy, dyz, dzx, dx2, dz2, st = range(10)
    assert B[s, s] == pytest.approx(V[T.SS], abs=1e-14)
    assert B[s, px] == pytest.approx(V[T.SP] / s3, abs=1e-14)
    assert B[px, s] == pytest.approx(-V[T.SP] / s3, abs=1e-14)
    assert B[st, py] == pytest.approx(V[T.SSTP] / s3, abs=1e-14)
    assert B[px, px] == pytest.approx(V[T.PPS] / 3 + 2 * V[T.PPP] / 3, abs=1e-14)
    assert B[px, py] == pytest.approx((V[T.PPS] - V[T.PPP]) / 3, abs=1e-14)
    assert B[s, dxy] == pytest.approx(V[T.SD] / s3, abs=1e-14)
    assert B[s, dz2] == pytest.approx(0.0, abs=1e-14)
    assert B[s, dx2] == pytest.approx(0.0, abs=1e-14)
    # E_{x,xy} = sqrt3 l^2 m V_pds + m(1-2l^2) V_pdp at l=m=n=1/sqrt3
    assert B[px, dxy] == pytest.approx(V[T.PDS] / 3 + V[T.PDP] / (3 * s3), abs=1e-14)
    # E_{x,yz} = sqrt3 lmn V_pds - 2 lmn V_pdp
    assert B[px, dyz] == pytest.approx(V[T.PDS] / 3 - 2 * V[T.PDP] / (3 * s3), abs=1e-14)
    assert B[dxy, px] == pytest.approx(-B[px, dxy], abs=1e-14)
    # E_{xy,xy} = 3l^2m^2 s + (l^2+m^2-4l^2m^2) p + (n^2+l^2m^2) d
    assert B[dxy, dxy] == pytest.approx(V[T.DDS] / 3 + 2 * V[T.DDP] / 9 + 4 * V[T.DDD] / 9, abs=1e-14)
    # E_{xy,yz} = 3lm^2n s + ln(1-4m^2) p + ln(m^2-1) d
    assert B[dxy, dyz] == pytest.approx(V[T.DDS] / 3 - V[T.DDP] / 9 - 2 * V[T.DDD] / 9, abs=1e-14)
    Bx = T.sk_block(T.MODEL_SP3D5S, V, [1, 0, 0])
    assert Bx[px, px] == pytest.approx(V[T.PPS], abs=1e-14)
    assert Bx[py, py] == pytest.approx(V[T.PPP], abs=1e-14)
    assert Bx[s, dx2] == pytest.approx(0.5 * s3 * V[T.SD], abs=1e-14)
    assert Bx[s, dz2] == pytest.approx(-0.5 * V[T.SD], abs=1e-14)
    assert Bx[dz2, dz2] == pytest.approx(0.25 * V[T.DDS] + 0.75 * V[T.DDD], abs=1e-14)
    assert Bx[dx2, dz2] == pytest.approx(-0.25 * s3 * V[T.DDS] + 0.25 * s3 * V[T.DDD], abs=1e-14)
    assert Bx[py, dxy] == pytest.approx(V[T.PDP], abs=1e-14)
    assert Bx[px, dx2] == pytest.approx(0.5 * s3 * V[T.PDS], abs=1e-14)


def test_sk_reverse_is_transpose_and_rotation_choice_free():
    rng = np.random.default_rng(1)
    V = rng.uniform(-3, 3, 14)
    for d in T.SLOT_DIRS:
        B = T.sk_block(T.MODEL_SP3D5S, V, d)
        Br = T.sk_block(T.MODEL_SP3D5S, V, -d)
        assert np.abs(Br - B.T).max() < 1e-13
        # another rotation taking z to d (extra turn about d) gives the same block
        R = T.rotation_to(d)
        c, s_ = np.cos(0.7), np.sin(0.7)
        Rz = np.array([[c, -s_, 0], [s_, c, 0], [0, 0, 1]])
        D = T.orbital_rep(T.MODEL_SP3D5S, R @ Rz)
        assert np.abs(D @ T.bond_block_z(T.MODEL_SP3D5S, V) @ D.T - B).max() < 1e-13


def test_gamma_closed_form_sp3s():
    """sp3s* bulk at Gamma: p-like triplets at E_p +- (4/3)(V_pps + 2 V_ppp)."""
    for n in (1, 2):
        p = _cube(n, model=W.MODEL_SP3S)
        H = T.hamiltonian(p).toarray()
        ev = np.linalg.eigvalsh(H)
        V = p.params["sk"][0][0]
        Ep = p.params["onsite"][0][1]
        for sgn in (1, -1):
            e = Ep + sgn * 4.0 / 3.0 * (V[T.PPS] + 2 * V[T.PPP])
            assert np.sum(np.abs(ev - e) < 1e-10) >= 3


def test_spin_orbit_spectrum():
    for delta in (0.044, 0.29):
        H = T.spin_orbit_block(T.MODEL_SP3S, delta)
        lam = 2 * delta / 3
        idx = [1, 2, 3, 6, 7, 8]
        ev = np.sort(np.linalg.eigvalsh(H[np.ix_(idx, idx)]))
        assert np.allclose(ev, [-lam, -lam, lam / 2, lam / 2, lam / 2, lam / 2], atol=1e-14)
        assert abs(np.trace(H)) < 1e-15
        assert np.abs(H - H.conj().T).max() == 0


@pytest.mark.parametrize("spin", [0, 1])
def test_passivation_trace_and_hybrid(spin):
    for d in T.SLOT_DIRS:
        h = T.hybrid_vector(T.MODEL_SP3D5S, d)
        assert np.dot(h, h) == pytest.approx(1.0, abs=1e-15)
    p0 = _cube(2, (0, 0, 0), model=W.MODEL_SP3D5S, spin=spin)
    p1 = _cube(2, (0, 0, 0), model=W.MODEL_SP3D5S, spin=spin, passivation=30.0)
    t0 = np.trace(T.hamiltonian(p0).toarray()).real
    t1 = np.trace(T.hamiltonian(p1).toarray()).real
    n_dang = 24 * 4 - 12
    assert t1 - t0 == pytest.approx(30.0 * n_dang * (2 if spin else 1), rel=1e-12)


@pytest.mark.parametrize("kw", [dict(model=W.MODEL_SP3S), dict(model=W.MODEL_SP3D5S, spin=1),
                                dict(model=W.MODEL_SP3D5S, strain=True, potential=0.3,
                                     kfrac=(0.1, -0.2, 0.3)),
                                dict(model=W.MODEL_SP3D5S, spin=1, passivation=30.0,
                                     periodic=(0, 0, 0), strain=True)])
def test_hermitian_and_traces(kw):
    p = _cube(2, **kw)
    blk = T.build_blocks(p)
    H = T.csr_hamiltonian(blk)
    assert abs(H - H.conj().T).max() < 1e-14
    Hd = H.toarray()
    tr = sum(np.trace(blk["onsite"][i]) for i in range(p.n_atoms))
    assert np.trace(Hd) == pytest.approx(tr, rel=1e-13)
    fro = np.sum(np.abs(blk["onsite"]) ** 2) + np.sum(np.abs(blk["bonds"]) ** 2)
    assert np.trace(Hd @ Hd).real == pytest.approx(fro, rel=1e-12)


@pytest.mark.parametrize("n,model,spin", [(1, W.MODEL_SP3S, 0), (2, W.MODEL_SP3S, 0),
                                          (1, W.MODEL_SP3D5S, 1)])
def test_bulk_folding(n, model, spin):
    """Spectrum of the periodic n^3 supercell at k_s equals the union of the
    bulk two-atom H(k) spectra over the 4n^3 folded k-points."""
    kf = np.array([0.13, -0.27, 0.41])
    p = _cube(n, model=model, spin=spin, kfrac=kf)
    H = T.hamiltonian(p).toarray()
    ev = np.sort(np.linalg.eigvalsh(H))
    L = 4.0 * n
    par = p.params
    bulk = []
    for i in range(2 * n):
        for j in range(2 * n):
            for l in range(n):
                k = 2 * np.pi * (kf + np.array([i, j, l])) / L
                Hk = T.bulk_hk(model, spin, par["onsite"][0], par["sk"][0][0], par["so_delta"][0], k)
                bulk.append(np.linalg.eigvalsh(Hk))
    bulk = np.sort(np.concatenate(bulk))
    assert bulk.shape == ev.shape
    assert np.abs(bulk - ev).max() < 1e-10


def test_time_reversal_real_model():
    """Without spin, H(-k) = conj(H(k)): identical spectra."""
    kf = np.array([0.2, 0.1, -0.35])
    a = np.linalg.eigvalsh(T.hamiltonian(_cube(2, kfrac=kf)).toarray())
    b = np.linalg.eigvalsh(T.hamiltonian(_cube(2, kfrac=-kf)).toarray())
    assert np.abs(a - b).max() < 1e-11


def test_hx_rows_match_csr():
    p = _cube(2, model=W.MODEL_SP3D5S, spin=1, strain=True, potential=0.2,
              kfrac=(0.1, 0.0, -0.2))
    H = T.hamiltonian(p)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(p.dim) + 1j * rng.standard_normal(p.dim)
    y = (H @ x).reshape(p.n_atoms, -1)
    atoms = [0, 5, 17, 63]
    assert np.abs(T.hx_rows(p, atoms, x) - y[atoms]).max() < 1e-12


def test_gap_table_entries_reproduce():
    """The stored gap-accepted seeds still give the stored bulk band edges
    (coarse recomputation with the oracle's bulk H(k))."""
    from oracle import gap_search as G
    t = W.gap_table()
    assert {"model1_spin0", "model1_spin1", "model0_spin0", "model0_spin1"} <= set(t)
    for key, e in t.items():
        par = W.draw_params(np.random.default_rng(e["seed"]), e["model"], e["spin"], 1)
        v, c = G.band_edges(par, G.kpoints(e["grid"]))
        assert c - v >= 0.5
        assert abs(e["vbm"] - v) < 1e-12 and abs(e["cbm"] - c) < 1e-12
        assert abs(e["mid"] - 0.5 * (e["vbm"] + e["cbm"])) < 1e-12


def test_paper_structure_size_44nm_silicon_cube():
    """The silicon cube of the 3-D decomposition test (80 unit cells per
    direction, 44 nm edge, about 4 million atoms) as the lattice generator
    and the oracle's sublattice rule produce it: 8 distinct atoms per
    conventional cell, half on each sublattice, 80 planes of cells along
    any axis (the 1-D decomposition limit), and an edge of 80 a."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "structure_sizes.json")))
    n = g["cells_per_axis"]
    pos = W.diamond_positions(n, n, n)
    assert pos.shape == (8 * n ** 3, 3)
    assert abs(pos.shape[0] - g["atoms_approx"]) <= g["atoms_rel_tol"] * g["atoms_approx"]
    key = (pos[:, 0].astype(np.int64) * (4 * n) + pos[:, 1]) * (4 * n) + pos[:, 2]
    assert np.unique(key).size == pos.shape[0]
    sub = T.sublattice(pos)
    assert int(sub.sum()) == pos.shape[0] // 2
    assert np.unique(pos[:, 2] // 4).size == g["max_1d_slabs"]
    assert abs(n * g["si_lattice_constant_nm"] - g["edge_nm"]) <= 0.02 * g["edge_nm"]
