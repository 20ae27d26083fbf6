"""Seeded synthetic workloads for the tight-binding hot path.

This module holds input data only: diamond-lattice atom positions, species
draws, random tight-binding parameter sets, bond-strain factors, on-site
potentials, donor sites, k-points and Lanczos start vectors.  It contains no
Hamiltonian, eigensolver, Poisson or network arithmetic, so both the HIP
library and the CPU oracle can consume the same arrays without sharing any
code of the method.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64) with a
fixed draw order per workload: parameters, species, strain, potential,
donors, k-points, start vector.

Lengths are integers in units of a/4 (a = 0.5431 nm, the Si lattice
constant), energies are eV.

The paper (Lee, Ryu, Jiang, Klimeck, "Million Atom Electronic Structure and
Device Calculations on Peta-Scale Computers") names the sp3s* and sp3d5s*
empirical tight-binding models (Abstract; Sec. I) but prints no parameter
table, so every parameter set here is synthetic: on-site energies uniform in
[-5, 12] eV per orbital type and two-centre integrals uniform in [-3, 3] eV.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

A_SI_NM = 0.5431          # Si conventional lattice constant (nm)
H_GRID_NM = A_SI_NM / 4   # grid spacing of the a/4 integer lattice (nm)

MODEL_SP3S = 0
MODEL_SP3D5S = 1

# canonical order of the 14 Slater-Koster two-centre integrals
SK_KEYS = ("ss_sigma", "s*s*_sigma", "ss*_sigma", "sp_sigma", "s*p_sigma",
           "sd_sigma", "s*d_sigma", "pp_sigma", "pp_pi", "pd_sigma", "pd_pi",
           "dd_sigma", "dd_pi", "dd_delta")
SK_USED_SP3S = (0, 1, 2, 3, 4, 7, 8)

# fcc offsets of the conventional cell (a/4 units); sublattice B = A + (1,1,1)
FCC_OFFSETS = np.array([[0, 0, 0], [0, 2, 2], [2, 0, 2], [2, 2, 0]], dtype=np.int32)


def n_orbitals(model: int, spin: int) -> int:
    """Orbitals per atom, spin included."""
    base = 5 if model == MODEL_SP3S else 10
    return base * (2 if spin else 1)


def diamond_positions(nx: int, ny: int, nz: int) -> np.ndarray:
    """Integer positions (a/4 units) of an nx*ny*nz block of conventional
    diamond cells, atom index = ((cz*ny + cy)*nx + cx)*8 + 2*f + s."""
    cz, cy, cx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cell = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1).astype(np.int32) * 4
    pos = np.empty((cell.shape[0], 4, 2, 3), dtype=np.int32)
    for f in range(4):
        pos[:, f, 0, :] = cell + FCC_OFFSETS[f]
        pos[:, f, 1, :] = cell + FCC_OFFSETS[f] + 1
    return pos.reshape(-1, 3)


def _draw_homopolar(rng, model):
    """One species' synthetic parameter set: on-site (E_s, E_p, E_d, E_s*) and
    the 14 two-centre integrals (unused ones zero for sp3s*)."""
    onsite = rng.uniform(-5.0, 12.0, size=4)
    sk = rng.uniform(-3.0, 3.0, size=14)
    if model == MODEL_SP3S:
        onsite[2] = 0.0
        mask = np.zeros(14, dtype=bool)
        mask[list(SK_USED_SP3S)] = True
        sk[~mask] = 0.0
    return onsite, sk


def draw_params(rng, model: int, spin: int, n_species: int = 1) -> dict:
    """Synthetic parameter sets for ``n_species`` species.

    Species are drawn independently; a bond between two different species
    uses the mean of the two homopolar sets (so sk[a][b] == sk[b][a]).
    Spin-orbit splittings Delta_so are uniform in [0, 0.1] eV when spin is on.
    """
    onsite = np.zeros((n_species, 4))
    homo = np.zeros((n_species, 14))
    for s in range(n_species):
        onsite[s], homo[s] = _draw_homopolar(rng, model)
    so = rng.uniform(0.0, 0.1, size=n_species) if spin else np.zeros(n_species)
    sk = 0.5 * (homo[:, None, :] + homo[None, :, :])
    return dict(model=model, spin=int(spin), n_species=n_species,
                onsite=onsite, sk=sk, so_delta=so, passivation_eV=0.0)


def draw_strain(rng, n_atoms: int) -> np.ndarray:
    """Per-bond hopping scale f = 1 + 0.01*g, g ~ N(0,1), one draw per
    undirected bond in canonical order (A-sublattice atom ascending, slot
    0..3).  Returned as [n_atoms][4]; rows of B-sublattice atoms (odd indices
    of the canonical order) hold 1.0 and are not read: a bond's reverse
    direction uses its A atom's factor."""
    out = np.ones((n_atoms, 4))
    n_a = n_atoms // 2
    g = rng.standard_normal((n_a, 4))
    out[0::2] = 1.0 + 0.01 * g
    return out


def draw_start_vector(rng, dim: int, complex_: bool) -> np.ndarray:
    """Lanczos start vector, uniform in [-1, 1); complex vectors interleave
    real and imaginary parts."""
    v = rng.uniform(-1.0, 1.0, size=dim * (2 if complex_ else 1))
    if complex_:
        return v[0::2] + 1j * v[1::2]
    return v


@dataclass
class Problem:
    """A tight-binding problem instance: geometry, parameters, per-bond and
    per-atom inputs, and Lanczos settings."""
    name: str
    pos_q: np.ndarray
    species: np.ndarray
    box_q: tuple
    periodic: tuple
    params: dict
    bond_scale: np.ndarray | None = None
    onsite_pot: np.ndarray | None = None
    kfrac: np.ndarray | None = None
    sigma: float = 0.0
    k: int = 8
    m: int = 300
    reorth: int = 1
    prec: str = "f64"
    v0: np.ndarray | None = None
    extra: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.pos_q.shape[0])

    @property
    def n_orb(self) -> int:
        return n_orbitals(self.params["model"], self.params["spin"])

    @property
    def dim(self) -> int:
        return self.n_atoms * self.n_orb

    @property
    def is_complex(self) -> bool:
        return bool(self.params["spin"]) or (self.kfrac is not None and np.any(self.kfrac != 0))


_GAP_TABLE = os.path.join(os.path.dirname(__file__), "gap_table.json")


def gap_table() -> dict:
    """Accepted parameter seeds with a bulk gap, written by the oracle's
    gap-search script (entries: model/spin -> seed, vbm, cbm, mid)."""
    if not os.path.exists(_GAP_TABLE):
        return {}
    with open(_GAP_TABLE) as f:
        return json.load(f)


def _gap_entry(model, spin):
    key = f"model{model}_spin{spin}"
    t = gap_table()
    if key not in t:
        raise KeyError(f"no gap-accepted parameter seed for {key}; run oracle/gap_search.py")
    return t[key]


def problem_periodic_cube(n: int, seed: int = 0, model=MODEL_SP3S, spin=0, prec="f64",
                          strain=False, potential=0.0, kfrac=None, sigma=1.0, k=8,
                          m=300, reorth=1, n_species=1, alloy_frac=0.0,
                          periodic=(1, 1, 1), nxyz=None, passivation=0.0,
                          param_seed=None) -> Problem:
    """Generic diamond block with the fixed draw order.

    ``param_seed`` (default ``seed``) seeds the parameter draw separately so a
    gap-accepted parameter set can be combined with any geometry seed."""
    nx, ny, nz = nxyz if nxyz is not None else (n, n, n)
    prng = np.random.default_rng(seed if param_seed is None else param_seed)
    params = draw_params(prng, model, spin, n_species)
    params["passivation_eV"] = float(passivation)
    rng = np.random.default_rng(seed + 7919)
    pos = diamond_positions(nx, ny, nz)
    N = pos.shape[0]
    if n_species > 1:
        species = (rng.random(N) < alloy_frac).astype(np.uint8)
    else:
        species = np.zeros(N, dtype=np.uint8)
    bond_scale = draw_strain(rng, N) if strain else None
    pot = rng.uniform(-potential, potential, size=N) if potential else None
    kf = None if kfrac is None else np.asarray(kfrac, dtype=np.float64)
    prob = Problem(name=f"cube{nx}x{ny}x{nz}", pos_q=pos, species=species,
                   box_q=(4 * nx, 4 * ny, 4 * nz), periodic=tuple(int(p) for p in periodic),
                   params=params, bond_scale=bond_scale, onsite_pot=pot, kfrac=kf,
                   sigma=float(sigma), k=k, m=m, reorth=reorth, prec=prec)
    prob.v0 = draw_start_vector(rng, prob.dim, prob.is_complex)
    return prob


# ---------------------------------------------------------------------------
# The five workloads.  Sizes follow the benchmarks the paper reports: its unit
# of cost is a fixed number of Lanczos iterations on a silicon block
# (Sec. II-B, Figs. 2-3), and the self-consistent application is a P
# delta-layer in Si at 4 K (Sec. III-B).
# ---------------------------------------------------------------------------

def c1_lanczos_fp64(seed: int = 0, n: int = 4) -> Problem:
    """Plain FP64 method: periodic Si block of n^3 conventional cells (512
    atoms at n=4), sp3s* without spin, Gamma point, 8 eigenvalues nearest
    1.0 eV, 300 iterations, full reorthogonalisation."""
    p = problem_periodic_cube(n, seed, model=MODEL_SP3S, spin=0, prec="f64",
                              sigma=1.0, k=8, m=300, reorth=1)
    p.name = f"c1_si{n}x{n}x{n}_sp3s_fp64"
    return p


def c2_hardwall_so(seed: int = 0, n: int = 20, m: int = 500) -> Problem:
    """FP32 H.x with FP64 Lanczos scalars: hard-wall Si cube of n^3 cells
    (64,000 atoms at n=20), sp3d5s* with spin-orbit (20 orbitals, complex
    Hermitian), dangling-bond hybrids shifted +30 eV, Gaussian +-1 % bond
    strain, 16 eigenvalues near mid-gap."""
    ge = _gap_entry(MODEL_SP3D5S, 1)
    p = problem_periodic_cube(n, seed, model=MODEL_SP3D5S, spin=1, prec="f32",
                              strain=True, periodic=(0, 0, 0), passivation=30.0,
                              sigma=ge["mid"], k=16, m=m, reorth=1,
                              param_seed=ge["seed"])
    p.extra["gap"] = ge
    p.name = f"c2_si{n}x{n}x{n}_sp3d5s_so_hardwall_fp32"
    return p


def c3_alloy(seed: int = 0, n: int = 51, m: int = 500) -> Problem:
    """Million-atom FP32 H.x: periodic random Si(0.7)Ge(0.3) alloy of n^3
    cells (1,061,208 atoms at n=51), sp3d5s* without spin (10 orbitals, real
    symmetric), 500 Lanczos iterations without reorthogonalisation."""
    p = problem_periodic_cube(n, seed, model=MODEL_SP3D5S, spin=0, prec="f32",
                              n_species=2, alloy_frac=0.3, sigma=0.0, k=16, m=m,
                              reorth=0)
    p.name = f"c3_si0.7ge0.3_{n}x{n}x{n}_sp3d5s_fp32"
    return p


def c4_batch(seed: int = 0, n_cells: int = 48, k_per_cell: int = 4, nrhs: int = 16,
             edge_range=(2, 12)) -> list:
    """Batched multi-vector H.X: ``n_cells`` periodic cubic cells with edges
    uniform in ``edge_range`` conventional cells, each at ``k_per_cell``
    seeded k-points (fractions uniform in [-0.5, 0.5)), sp3s* with spin-orbit
    (10x10 complex blocks), ``nrhs`` seeded complex right-hand vectors.  One
    shared parameter set.  Returns a list of (Problem, X) pairs."""
    rng = np.random.default_rng(seed)
    params = draw_params(rng, MODEL_SP3S, 1, 1)
    edges = rng.integers(edge_range[0], edge_range[1] + 1, size=n_cells)
    out = []
    for c, e in enumerate(edges):
        pos = diamond_positions(int(e), int(e), int(e))
        N = pos.shape[0]
        for kk in range(k_per_cell):
            kf = rng.uniform(-0.5, 0.5, size=3)
            prob = Problem(name=f"c4_cell{c}_n{e}_k{kk}", pos_q=pos,
                           species=np.zeros(N, dtype=np.uint8), box_q=(4 * e,) * 3,
                           periodic=(1, 1, 1), params=params, kfrac=kf, prec="f32")
            x = rng.uniform(-1, 1, size=(N * 10, nrhs)) + 1j * rng.uniform(-1, 1, size=(N * 10, nrhs))
            out.append((prob, x))
    return out


def c5_slab(seed: int = 0, nx: int = 8, ny: int = 8, nz: int = 60, n_donors: int = 64) -> Problem:
    """Schrodinger-Poisson slab: (001) delta-doped Si slab of nx*ny*nz cells
    (30,720 atoms at 8x8x60), periodic in x,y and hard-wall in z with
    dangling-bond hybrids shifted +30 eV, sp3d5s* without spin.  ``n_donors``
    donor ions on distinct atoms of the mid-slab (001) plane."""
    ge = _gap_entry(MODEL_SP3D5S, 0)
    p = problem_periodic_cube(0, seed, model=MODEL_SP3D5S, spin=0, prec="f32",
                              periodic=(1, 1, 0), nxyz=(nx, ny, nz), passivation=30.0,
                              sigma=ge["cbm"], k=48, m=600, reorth=1,
                              param_seed=ge["seed"])
    rng = np.random.default_rng(seed + 104729)
    donors = draw_donor_sites(rng, p.pos_q, plane_qz=2 * nz, n_donors=n_donors)
    p.extra.update(gap=ge, donor_atoms=donors, grid=(4 * nx, 4 * ny, 4 * nz))
    p.name = f"c5_slab{nx}x{ny}x{nz}_sp3d5s"
    return p


def draw_donor_sites(rng, pos_q: np.ndarray, plane_qz: int, n_donors: int) -> np.ndarray:
    """Distinct donor atoms drawn from the atoms of the (001) plane
    z = plane_qz (a/4 units), returned sorted by atom index."""
    sites = np.flatnonzero(pos_q[:, 2] == plane_qz)
    if n_donors > sites.size:
        raise ValueError("more donors than sites in the plane")
    pick = rng.choice(sites.size, size=n_donors, replace=False)
    return np.sort(sites[pick]).astype(np.int32)


def sublattice_masks(pos_q: np.ndarray, grid: tuple) -> np.ndarray:
    """[2][nz][ny][nx] float32: 1 on the grid nodes holding an A-sublattice
    (first map) or B-sublattice (second map) atom."""
    nx, ny, nz = grid
    m = np.zeros((2, nz, ny, nx), dtype=np.float32)
    q = np.asarray(pos_q)
    sub = (q.sum(axis=1) % 4 == 3).astype(np.int64)
    m[sub, q[:, 2], q[:, 1], q[:, 0]] = 1.0
    return m


def donor_map(pos_q: np.ndarray, donor_atoms: np.ndarray, grid: tuple) -> np.ndarray:
    """Donor-count map on the a/4 grid, shape [nz][ny][nx] (float32)."""
    nx, ny, nz = grid
    m = np.zeros((nz, ny, nx), dtype=np.float32)
    q = pos_q[donor_atoms]
    np.add.at(m, (q[:, 2], q[:, 1], q[:, 0]), 1.0)
    return m


CONFIGS = {
    "c1": c1_lanczos_fp64,
    "c2": c2_hardwall_so,
    "c3": c3_alloy,
    "c4": c4_batch,
    "c5": c5_slab,
}


# ---------------------------------------------------------------------------
# Schrodinger-Poisson study slab and surrogate initialisation
# ---------------------------------------------------------------------------

STUDY_SLAB = dict(nx=3, ny=3, nz=8, n_donors=9)


def study_slab(seed: int) -> Problem:
    """Delta-doped slab used for the start-potential study: 3x3x8 cells
    (576 atoms), 9 donors on the mid (001) plane (half a monolayer, the same
    areal density as the 8x8x60-cell slab with 64 donors), same parameters
    and geometry for every seed; only the donor layout and start vector
    change with the seed."""
    return c5_slab(seed, **STUDY_SLAB)


def init_surrogate_weights(seed: int, channels: int = 32, in_channels: int = 1, n_layers: int = 4) -> np.ndarray:
    """He-normal initial weights of the 3x3x3 layers (c_in->C->...->C->1),
    zero biases, flattened in canonical order W[co][ci][dz][dy][dx], b[co]."""
    rng = np.random.default_rng(seed)
    out = []
    shapes = [(channels, in_channels)] + [(channels, channels)] * (n_layers - 2) + [(1, channels)]
    for co, ci in shapes:
        std = np.sqrt(2.0 / (27 * ci))
        out.append((rng.standard_normal(co * ci * 27) * std).astype(np.float32))
        out.append(np.zeros(co, np.float32))
    return np.concatenate(out)
