"""Host logic of the library (no GPU): the C ABI loads and exports every
declared symbol, the neighbour table is bit-exact against the oracle's
search, and the assembled FP64 blocks (closed-form Slater-Koster table)
match the oracle's rotation-built blocks."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1003_4570_amd as tbh
import workloads as W
from oracle import tb as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "tbh.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tbh_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = tbh.lib()
    decl = _declared_symbols()
    assert len(decl) >= 10
    for name in decl:
        assert hasattr(L, name), name
        assert name in tbh.exported_symbols(), name
    assert tbh.version() >= 100


CASES = [
    dict(n=2, model=W.MODEL_SP3S),
    dict(n=2, model=W.MODEL_SP3D5S, strain=True, potential=0.4),
    dict(n=2, model=W.MODEL_SP3D5S, spin=1, periodic=(0, 0, 0), passivation=30.0, strain=True),
    dict(n=2, model=W.MODEL_SP3S, spin=1, kfrac=(0.1, -0.3, 0.25)),
    dict(n=2, model=W.MODEL_SP3D5S, periodic=(1, 1, 0), passivation=30.0, kfrac=(0.2, 0.1, 0.0)),
    dict(n=3, model=W.MODEL_SP3D5S, n_species=2, alloy_frac=0.3),
]


@pytest.mark.parametrize("case", CASES)
def test_blocks_match_oracle(case):
    c = dict(case)
    n = c.pop("n")
    p = W.problem_periodic_cube(n, seed=7, **c)
    nbr, wrap, on, bd, cplx = tbh.build_blocks_host(**tbh.problem_args(p))
    blk = T.build_blocks(p)
    assert np.array_equal(nbr, blk["nbr"])
    assert np.array_equal(wrap, blk["wrap"])
    assert cplx == blk["complex"]
    assert np.abs(on - blk["onsite"]).max() < 1e-13
    assert np.abs(bd - blk["bonds"]).max() < 1e-13
    # bitwise Hermitian: B_jb == B_ib^H for j = nbr(i,b); on-site Hermitian
    for b in range(4):
        ok = nbr[:, b] >= 0
        i = np.flatnonzero(ok)
        j = nbr[ok, b]
        assert np.array_equal(bd[j, b], np.conj(np.swapaxes(bd[i, b], -1, -2)))
    assert np.array_equal(on, np.conj(np.swapaxes(on, -1, -2)))


def test_sk_closed_form_vs_rotation_random_directions():
    """The library's closed-form table against the rotation construction at
    the 8 bond directions and with random parameters (through the builder)."""
    for seed in range(4):
        p = W.problem_periodic_cube(1, seed=seed, model=W.MODEL_SP3D5S)
        _, _, _, bd, _ = tbh.build_blocks_host(**tbh.problem_args(p))
        blk = T.build_blocks(p)
        assert np.abs(bd - blk["bonds"]).max() < 1e-13


def _geom_args(p, **over):
    a = tbh.problem_args(p)
    a.update(over)
    return a


def test_invalid_geometry_rejected():
    p = W.problem_periodic_cube(1, seed=1)
    bad = p.pos_q.copy()
    bad[3] = bad[2]
    with pytest.raises(tbh.TBHError) as e:
        tbh.build_blocks_host(**_geom_args(p, pos_q=bad))
    assert e.value.code == tbh.TBH_EINVAL and "duplicate" in str(e.value)
    bad = p.pos_q.copy()
    bad[0] = (1, 0, 0)
    with pytest.raises(tbh.TBHError) as e:
        tbh.build_blocks_host(**_geom_args(p, pos_q=bad))
    assert "diamond" in str(e.value)
    bad = p.pos_q.copy()
    bad[0] = (40, 0, 0)
    with pytest.raises(tbh.TBHError):
        tbh.build_blocks_host(**_geom_args(p, pos_q=bad))
    spc = p.species.copy()
    spc[0] = 3
    with pytest.raises(tbh.TBHError) as e:
        tbh.build_blocks_host(**_geom_args(p, species=spc))
    assert "species" in str(e.value)
    sk = np.array(p.params["sk"]).copy()
    with pytest.raises(tbh.TBHError):
        tbh.build_blocks_host(**_geom_args(p, model=7))
    with pytest.raises(tbh.TBHError):
        tbh.build_blocks_host(**_geom_args(p, box_q=(6, 4, 4)))


def test_hardwall_dangling_and_reverse_slot():
    for n in (1, 2, 3):
        p = W.problem_periodic_cube(n, seed=2, periodic=(0, 0, 0))
        nbr, wrap, _, _, _ = tbh.build_blocks_host(**tbh.problem_args(p))
        assert int((nbr < 0).sum()) == 24 * n * n - 6 * n
        for b in range(4):
            ok = nbr[:, b] >= 0
            assert np.array_equal(nbr[nbr[ok, b], b], np.flatnonzero(ok))


def test_study_slab_input_maps():
    """Surrogate input maps of the study slab: the two sublattice masks are
    disjoint, hold one atom each per occupied node (half the atoms each),
    and an A node plus (1,1,1) is a B node; the donor map counts the donors."""
    p = W.study_slab(3)
    g = p.extra["grid"]
    m = W.sublattice_masks(p.pos_q, g)
    assert m.shape == (2, g[2], g[1], g[0])
    assert m[0].sum() == m[1].sum() == p.pos_q.shape[0] // 2
    assert (m[0] * m[1]).sum() == 0
    za, ya, xa = np.nonzero(m[0])
    inside = za + 1 < g[2]
    assert np.all(m[1][za[inside] + 1, (ya[inside] + 1) % g[1], (xa[inside] + 1) % g[0]] == 1)
    d = W.donor_map(p.pos_q, p.extra["donor_atoms"], g)
    assert d.sum() == len(p.extra["donor_atoms"])
    assert np.all((d > 0) <= (m[0] + m[1] > 0))


def test_lattice_shifts_are_symmetries_of_the_study_slab():
    """The in-plane translations used for the surrogate's symmetrized mean
    and augmentation map the atom set and the donor-plane site set of the
    study slab onto themselves; a symmetrized map is invariant under them."""
    from paper_1003_4570_amd import surrogate as S
    p = W.study_slab(0)
    g = p.extra["grid"]
    sh = S.lattice_shifts(g)
    assert len(sh) == 18 and (0, 0) in sh
    atoms = set(map(tuple, p.pos_q.tolist()))
    for sx, sy in sh:
        moved = {((x + sx) % g[0], (y + sy) % g[1], z) for x, y, z in atoms}
        assert moved == atoms
    rng = np.random.default_rng(0)
    a = rng.standard_normal((g[2], g[1], g[0]))
    s = S.symmetrize(a, g)
    for sx, sy in sh:
        assert np.allclose(np.roll(s, (sy, sx), axis=(-2, -1)), s)
    assert np.isclose(s.mean(), a.mean())


def test_point_ops_are_symmetries_of_the_study_slab():
    """The in-plane point operations averaged over by the surrogate map the
    study slab's atoms and its donor-plane sites onto themselves (each
    sublattice onto itself) and are involutions."""
    import torch
    from paper_1003_4570_amd import surrogate as S
    p = W.study_slab(0)
    g = p.extra["grid"]
    m = torch.from_numpy(W.sublattice_masks(p.pos_q, g))
    plane = torch.zeros_like(m[0])
    for s in range(60):
        d = W.donor_map(W.study_slab(s).pos_q, W.study_slab(s).extra["donor_atoms"], g)
        plane += torch.from_numpy(d > 0).float()
    sites = plane > 0
    ops = S.point_ops()
    assert len(ops) == 4
    a = torch.randn(3, g[2], g[1], g[0], dtype=torch.float64)
    for op, inv in ops:
        assert torch.equal(op(m), m)
        assert torch.equal(op(sites), sites)
        assert torch.equal(inv(op(a)), a)


TAB_HOST_CASES = [
    dict(n=2, model=W.MODEL_SP3S),
    dict(n=3, model=W.MODEL_SP3D5S, n_species=2, alloy_frac=0.3, potential=0.4),
    dict(n=2, model=W.MODEL_SP3D5S, periodic=(0, 0, 0)),
    dict(n=0, nxyz=(2, 2, 5), model=W.MODEL_SP3D5S, n_species=2, alloy_frac=0.5, periodic=(1, 1, 0)),
]


@pytest.mark.parametrize("case", TAB_HOST_CASES)
def test_tabulated_table_and_keys_match_oracle_blocks(case):
    """The table of distinct bond blocks and the per-atom key records against
    the oracle's blocks, built bond by bond from each bond's own direction:
    every bond's looked-up block equals its block, dangling slots are marked,
    the key is a function of (sublattice, species pair, slot), every entry is
    used, and the on-site diagonals equal the on-site blocks less the
    potential."""
    c = dict(case)
    n = c.pop("n")
    p = W.problem_periodic_cube(n, seed=7, **c)
    blocks, diag, keys = tbh.tabulate_host(**tbh.problem_args(p, tabulated=True))
    blk = T.build_blocks(p)
    nbr, no, N = blk["nbr"], blk["n_o"], p.n_atoms
    spc = np.asarray(p.species, dtype=np.int64)
    assert np.array_equal(keys[:, :4] == 255, nbr < 0)
    assert np.array_equal(keys[:, 4], spc)
    assert not keys[:, 5:].any()
    i, b = np.nonzero(nbr >= 0)
    k = keys[i, b].astype(np.int64)
    assert np.array_equal(np.unique(k), np.arange(blocks.shape[0]))
    assert np.abs(blocks[k] - blk["bonds"][i, b]).max() < 1e-13
    sub = T.sublattice(p.pos_q)
    cls = ((sub[i] * 4 + spc[i]) * 4 + spc[nbr[i, b]]) * 4 + b
    for c_ in np.unique(cls):
        assert np.unique(k[cls == c_]).size == 1
    U = np.zeros(N) if p.onsite_pot is None else np.asarray(p.onsite_pot, dtype=np.float64)
    D = np.zeros((N, no, no))
    D[:, np.arange(no), np.arange(no)] = diag[spc]
    assert np.abs(blk["onsite"] - U[:, None, None] * np.eye(no) - D).max() < 1e-13


@pytest.mark.parametrize("bad", [dict(strain=True), dict(spin=1), dict(kfrac=(0.1, 0.2, 0.0)),
                                 dict(periodic=(0, 0, 0), passivation=30.0)])
def test_tabulate_refuses_what_a_table_cannot_hold(bad):
    p = W.problem_periodic_cube(2, seed=3, model=W.MODEL_SP3S, **bad)
    with pytest.raises(tbh.TBHError):
        tbh.tabulate_host(**tbh.problem_args(p, tabulated=True))
