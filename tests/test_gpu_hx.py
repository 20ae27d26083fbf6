"""GPU parity of the block H.x kernels against the oracle's scalar CSR H.x.

Bar: FP64 relative 2-norm error <= 1e-12; FP32 <= 1e-5 (the FP32 input x is
applied by the oracle in FP64, so the error is the kernel's storage and
accumulation rounding: about sqrt(K) * 2^-24 for K <= 100 terms per row).
"""
import numpy as np
import pytest

import paper_1003_4570_amd as tbh
import workloads as W
from oracle import tb as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return tbh.Context(0)


def _rand_x(p, rng, cplx, dtype):
    import torch
    x = rng.uniform(-1, 1, p.dim) + (1j * rng.uniform(-1, 1, p.dim) if cplx else 0)
    xt = torch.tensor(x).to(dtype)
    return x, xt


def _run(ctx, p, prec, lanes=0, seed=0):
    import torch
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec=prec, lanes_per_atom=lanes))
    rng = np.random.default_rng(seed)
    dt = h.torch_dtype()
    x, xt = _rand_x(p, rng, h.is_complex, dt)
    xd = xt.cuda()
    y = tbh.apply_h(h, xd)
    y2 = tbh.apply_h(h, xd)
    torch.cuda.synchronize()
    assert torch.equal(y, y2), "H.x not bitwise deterministic"
    H = T.hamiltonian(p)
    xr = xt.numpy().astype(np.complex128 if h.is_complex else np.float64)
    yr = H @ xr
    yg = y.cpu().numpy().astype(np.complex128 if h.is_complex else np.float64)
    row_bound_check(H, xr, yg, yr, prec)
    return np.linalg.norm(yg - yr) / np.linalg.norm(yr), h


def row_bound_check(H, x, y, yr, prec):
    """Per-row forward error bound of a dot product: |y_i - y_ref,i| <=
    (K + 1) u (|H| |x|)_i with K the terms of row i (K-term summation) plus
    one rounding of each stored element, u the unit roundoff (2^-24 FP32,
    2^-53 FP64).  A single wrong row fails it even when the normwise error
    stays small."""
    import scipy.sparse as sp
    A = abs(sp.csr_matrix(H))
    K = np.diff(A.indptr)
    u = 2.0 ** -53 if prec == "f64" else 2.0 ** -24
    # complex rows: a complex product is 4 real products and 2 sums
    c = 2.0 if np.iscomplexobj(H) else 1.0
    bound = c * (K + 1) * u * (A @ np.abs(x)) + 1e-300
    ratio = np.abs(y - yr) / bound
    assert ratio.max() <= 1.0, (prec, float(ratio.max()), int(np.argmax(ratio)))


CASES = [
    ("sp3s_periodic", dict(n=2, model=W.MODEL_SP3S)),
    ("sp3s_ragged", dict(n=3, model=W.MODEL_SP3S, strain=True, potential=0.3)),
    ("sp3d5s_alloy", dict(n=3, model=W.MODEL_SP3D5S, n_species=2, alloy_frac=0.3)),
    ("sp3d5s_kpoint", dict(n=2, model=W.MODEL_SP3D5S, kfrac=(0.1, -0.2, 0.3))),
    ("sp3s_so_k", dict(n=3, model=W.MODEL_SP3S, spin=1, kfrac=(0.3, 0.1, -0.4))),
    ("sp3d5s_so_hardwall", dict(n=2, model=W.MODEL_SP3D5S, spin=1, periodic=(0, 0, 0),
                                passivation=30.0, strain=True)),
    ("slab", dict(n=0, nxyz=(2, 2, 5), model=W.MODEL_SP3D5S, periodic=(1, 1, 0), passivation=30.0)),
]


@pytest.mark.parametrize("name,case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_hx_parity(ctx, name, case, prec):
    c = dict(case)
    n = c.pop("n")
    p = W.problem_periodic_cube(n, seed=11, **c)
    print(f"case={name} prec={prec} atoms={p.n_atoms}", flush=True)
    err, h = _run(ctx, p, prec)
    tol = 1e-12 if prec == "f64" else 1e-5
    assert err <= tol, (name, prec, err)


@pytest.mark.parametrize("no_model,spin,lanes", [(W.MODEL_SP3S, 0, 1), (W.MODEL_SP3S, 0, 5),
                                                 (W.MODEL_SP3D5S, 0, 1), (W.MODEL_SP3D5S, 0, 2),
                                                 (W.MODEL_SP3D5S, 0, 5), (W.MODEL_SP3D5S, 1, 1),
                                                 (W.MODEL_SP3D5S, 1, 2), (W.MODEL_SP3D5S, 1, 5)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_hx_every_lane_shape(ctx, no_model, spin, lanes, prec):
    p = W.problem_periodic_cube(2, seed=5, model=no_model, spin=spin, strain=True,
                                kfrac=(0.05, 0.1, 0.0) if spin else None)
    print(f"model={no_model} spin={spin} lanes={lanes} prec={prec}", flush=True)
    err, h = _run(ctx, p, prec, lanes=lanes)
    assert h.info["lanes_per_atom"] == lanes
    assert err <= (1e-12 if prec == "f64" else 1e-5)


def test_hx_potential_update(ctx):
    import torch
    p = W.problem_periodic_cube(2, seed=3, model=W.MODEL_SP3D5S, potential=0.0)
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec="f64"))
    rng = np.random.default_rng(1)
    U = rng.uniform(-0.5, 0.5, p.n_atoms)
    tbh.ham_set_potential(h, torch.tensor(U).cuda())
    x = rng.uniform(-1, 1, p.dim)
    y = tbh.apply_h(h, torch.tensor(x).cuda()).cpu().numpy()
    p.onsite_pot = U
    yr = T.hamiltonian(p) @ x
    assert np.linalg.norm(y - yr) / np.linalg.norm(yr) < 1e-12
    tbh.ham_set_potential(h, None)
    p.onsite_pot = None
    y0 = tbh.apply_h(h, torch.tensor(x).cuda()).cpu().numpy()
    assert np.linalg.norm(y0 - T.hamiltonian(p) @ x) / np.linalg.norm(y0) < 1e-12


FORMATS = [("stored_f64", dict(prec="f64")), ("stored_f32", dict(prec="f32", keep_f64=True)),
           ("tabulated_f64", dict(prec="f64", tabulated=True)),
           ("tabulated_f32", dict(prec="f32", tabulated=True, keep_f64=True)),
           ("multi_vector", dict(prec="f32", multi_vector=True))]


@pytest.mark.parametrize("name,kw", FORMATS, ids=[f[0] for f in FORMATS])
def test_set_potential_same_rule_every_format(ctx, name, kw):
    """The build-time potential is the ham's per-atom potential in every
    storage format: H = H_TB + U_build after the build, H_TB + U after
    tbh_ham_set_potential(U), H_TB after set_potential(NULL); checked through
    the main copy, the FP64 copy and the multi-vector copy."""
    import torch
    p = W.problem_periodic_cube(3, seed=7, model=W.MODEL_SP3D5S, n_species=2, alloy_frac=0.4,
                                potential=0.5)
    u_build = p.onsite_pot.copy()
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, **kw))
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, p.dim)
    f32 = kw["prec"] == "f32"
    tol = 1e-5 if f32 else 1e-12
    xq = x.astype(np.float32).astype(np.float64) if f32 else x

    def check(pot):
        q = W.problem_periodic_cube(3, seed=7, model=W.MODEL_SP3D5S, n_species=2, alloy_frac=0.4)
        q.onsite_pot = pot
        H = T.hamiltonian(q)
        if kw.get("multi_vector"):
            X = np.repeat(xq[:, None], 16, axis=1)
            Y = tbh.apply_h_multi(h, torch.tensor(X, dtype=torch.float32).cuda()).cpu().numpy()
            y = Y[:, 5].astype(np.float64)
        else:
            y = tbh.apply_h(h, torch.tensor(xq, dtype=h.torch_dtype()).cuda()).cpu().numpy().astype(np.float64)
        yr = H @ xq
        assert np.linalg.norm(y - yr) / np.linalg.norm(yr) <= tol, (name, "main")
        if kw.get("keep_f64"):
            y64 = tbh.apply_h_f64(h, torch.tensor(x).cuda()).cpu().numpy()
            assert np.linalg.norm(y64 - H @ x) / np.linalg.norm(H @ x) <= 1e-12, (name, "f64 copy")

    check(u_build)
    U = rng.uniform(-0.3, 0.3, p.n_atoms)
    tbh.ham_set_potential(h, torch.tensor(U).cuda())
    check(U)
    tbh.ham_set_potential(h, None)
    check(None)


def test_hx_f64_copy_of_f32_ham(ctx):
    import torch
    p = W.problem_periodic_cube(2, seed=9, model=W.MODEL_SP3D5S, spin=1, periodic=(0, 0, 0),
                                passivation=30.0, strain=True)
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec="f32", keep_f64=True))
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, p.dim) + 1j * rng.uniform(-1, 1, p.dim)
    y = tbh.apply_h_f64(h, torch.tensor(x).cuda()).cpu().numpy()
    yr = T.hamiltonian(p) @ x
    assert np.linalg.norm(y - yr) / np.linalg.norm(yr) < 1e-12


@pytest.mark.parametrize("tab", [False, True], ids=["stored", "tabulated"])
def test_hx_c3_full_size_sampled(ctx, tab):
    """Million-atom alloy (51^3 cells, FP32, the measured configuration):
    sampled rows against the oracle computed atom by atom.  The tabulated
    format runs here with more tiles than resident blocks (each block walks
    several units); its Lanczos coefficients match the stored format's."""
    import torch
    p = W.c3_alloy(0)
    print(f"c3 atoms={p.n_atoms} tabulated={tab}", flush=True)
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, tabulated=tab))
    assert h.info["n_atoms"] == 1_061_208 and h.info["tabulated"] == int(tab)
    rng = np.random.default_rng(4)
    x = torch.empty(h.dim, dtype=torch.float32).uniform_(-1, 1, generator=torch.Generator().manual_seed(4))
    y = tbh.apply_h(h, x.cuda()).cpu().numpy()
    atoms = np.concatenate([[0, 1, p.n_atoms - 1], rng.integers(0, p.n_atoms, 400)])
    nbr, wrap = T.find_neighbours(p.pos_q, p.box_q, p.periodic)
    lnbr, lwrap = tbh.ham_neighbours(h)
    assert np.array_equal(nbr, lnbr) and np.array_equal(wrap, lwrap)
    ref = T.hx_rows(p, atoms, x.numpy().astype(np.float64), nbr=nbr, wrap=wrap)
    got = y.reshape(p.n_atoms, -1)[atoms]
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5
    # per row: (K + 1) u (|H||x|)_i with K = 41 terms (diagonal on-site + 4 blocks of 10)
    absref = T.hx_rows(p, atoms, np.abs(x.numpy().astype(np.float64)), nbr=nbr, wrap=wrap, absolute=True)
    assert (np.abs(got - ref) <= 42 * 2.0 ** -24 * absref + 1e-300).all()
    if tab:
        v0 = np.random.default_rng(5).uniform(-1, 1, h.dim)
        a1, b1, _ = tbh.lanczos_run(h, 8, v0, reorth=False)
        del h
        hs = tbh.build_hamiltonian(ctx, **tbh.problem_args(p))
        a2, b2, _ = tbh.lanczos_run(hs, 8, v0, reorth=False)
        assert np.abs(a1 - a2).max() < 1e-5 and np.abs(b1 - b2).max() < 1e-5


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_caller_order_does_not_matter(ctx, prec):
    """The library renumbers atoms into its stream order internally, so the
    same structure given with its atoms shuffled yields bitwise the same
    H.x (rows shuffled alike) and the same Lanczos coefficients."""
    import dataclasses
    import torch
    p = W.problem_periodic_cube(3, seed=4, model=W.MODEL_SP3D5S, strain=True, potential=0.4, prec=prec)
    rng = np.random.default_rng(11)
    perm = rng.permutation(p.n_atoms)
    q = dataclasses.replace(p, pos_q=p.pos_q[perm], species=p.species[perm],
                            bond_scale=None if p.bond_scale is None else p.bond_scale[perm],
                            onsite_pot=None if p.onsite_pot is None else p.onsite_pot[perm])
    no = p.n_orb
    h1 = tbh.build_hamiltonian(ctx, **tbh.problem_args(p))
    h2 = tbh.build_hamiltonian(ctx, **tbh.problem_args(q))
    x1 = torch.from_numpy(rng.uniform(-1, 1, (p.n_atoms, no))).to(h1.torch_dtype()).cuda()
    x2 = x1[torch.from_numpy(perm).cuda()].contiguous()
    y1 = tbh.apply_h(h1, x1.reshape(-1)).reshape(p.n_atoms, no)
    y2 = tbh.apply_h(h2, x2.reshape(-1)).reshape(p.n_atoms, no)
    assert torch.equal(y1[torch.from_numpy(perm).cuda()], y2)
    v0 = rng.uniform(-1, 1, (p.n_atoms, no))
    a1, b1, _ = tbh.lanczos_run(h1, 60, v0.ravel(), reorth=False)
    a2, b2, _ = tbh.lanczos_run(h2, 60, v0[perm].ravel(), reorth=False)
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)


TAB_CASES = [
    ("sp3s_periodic", dict(n=2, model=W.MODEL_SP3S)),
    ("sp3s_ragged_pot", dict(n=3, model=W.MODEL_SP3S, potential=0.3)),
    ("sp3d5s_alloy", dict(n=3, model=W.MODEL_SP3D5S, n_species=2, alloy_frac=0.3)),
    ("sp3d5s_alloy_pot", dict(n=3, model=W.MODEL_SP3D5S, n_species=2, alloy_frac=0.5, potential=0.4)),
    ("sp3d5s_hardwall", dict(n=2, model=W.MODEL_SP3D5S, periodic=(0, 0, 0))),
    ("slab_unpassivated", dict(n=0, nxyz=(2, 2, 5), model=W.MODEL_SP3D5S, periodic=(1, 1, 0))),
]


@pytest.mark.parametrize("name,case", TAB_CASES, ids=[c[0] for c in TAB_CASES])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_tabulated_hx_parity(ctx, name, case, prec):
    """Tabulated bond blocks (one table entry per sublattice, species pair
    and slot, checked against every atom's blocks at build time) against
    the oracle's CSR H.x; the FP64 copy of an FP32 ham too."""
    import torch
    kw = dict(case)
    n = kw.pop("n")
    p = W.problem_periodic_cube(n, seed=9, prec=prec, **kw)
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, tabulated=True, keep_f64=(prec == "f32")))
    assert h.info["tabulated"] == 1
    stored = tbh.build_hamiltonian(ctx, **tbh.problem_args(p))
    assert h.info["hx_bytes"] < 0.2 * stored.info["hx_bytes"] or p.n_orb == 5
    rng = np.random.default_rng(1)
    x, xt = _rand_x(p, rng, False, h.torch_dtype())
    y = tbh.apply_h(h, xt.cuda())
    H = T.hamiltonian(p)
    yr = H @ xt.numpy().astype(np.float64)
    err = np.linalg.norm(y.cpu().numpy().astype(np.float64) - yr) / np.linalg.norm(yr)
    assert err <= (1e-12 if prec == "f64" else 1e-5), err
    if prec == "f32":
        xd = torch.tensor(x, dtype=torch.float64).cuda()
        y64 = tbh.apply_h_f64(h, xd).cpu().numpy()
        assert np.linalg.norm(y64 - H @ x) / np.linalg.norm(H @ x) <= 1e-12


@pytest.mark.parametrize("bad", [dict(strain=True), dict(spin=1), dict(kfrac=(0.1, 0.2, 0.0)),
                                 dict(periodic=(0, 0, 0), passivation=30.0)])
def test_tabulated_rejects_what_a_table_cannot_hold(ctx, bad):
    p = W.problem_periodic_cube(2, seed=3, model=W.MODEL_SP3S, **bad)
    with pytest.raises(tbh.TBHError):
        tbh.build_hamiltonian(ctx, **tbh.problem_args(p, tabulated=True))


def test_tabulated_lanczos_c1(ctx):
    """C1 eigenvalues through the tabulated format: the same 8 distinct
    values nearest sigma as dense eigh (FP64, refined to 1e-9 eV), and the
    Lanczos coefficients equal the stored format's to rounding."""
    p = W.c1_lanczos_fp64(0)
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, tabulated=True))
    r = tbh.lanczos_eigs(h, p.sigma, p.k, p.m, p.v0, reorth=True)
    ev = np.linalg.eigvalsh(T.hamiltonian(p).toarray())
    u = [ev[0]]
    for e in ev[1:]:
        if e - u[-1] > 1e-8:
            u.append(e)
    u = np.array(u)
    want = np.sort(u[np.argsort(np.abs(u - p.sigma), kind="stable")[:p.k]])
    assert r["report"]["n_found"] == p.k
    assert np.abs(r["refined"] - want).max() < 1e-9
    hs = tbh.build_hamiltonian(ctx, **tbh.problem_args(p))
    a1, b1, _ = tbh.lanczos_run(h, 30, p.v0, reorth=False)
    a2, b2, _ = tbh.lanczos_run(hs, 30, p.v0, reorth=False)
    assert np.abs(a1 - a2).max() < 1e-10 and np.abs(b1 - b2).max() < 1e-10


SD_CASES = [
    ("sp3d5s_so_hardwall_strain", dict(n=2, model=W.MODEL_SP3D5S, spin=1, periodic=(0, 0, 0), passivation=30.0,
                                       strain=True)),
    ("sp3d5s_so_periodic_potential", dict(n=2, model=W.MODEL_SP3D5S, spin=1, potential=0.3)),
    ("sp3s_so_ragged", dict(n=3, model=W.MODEL_SP3S, spin=1, strain=True, periodic=(1, 1, 0), passivation=30.0)),
]


@pytest.mark.parametrize("name,case", SD_CASES, ids=[c[0] for c in SD_CASES])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_spin_diagonal_hx_parity(ctx, name, case, prec):
    """Spin-diagonal bond storage (I_2 (x) real block per bond, full complex
    on-site block) against the oracle's CSR H.x: FP64 <= 1e-12 and FP32 <=
    1e-5 relative plus the per-row rounding bound; the FP64 copy of an FP32
    ham <= 1e-12; bitwise the same as the stored format in FP64 is not
    required (the sums run in another order), the bytes are."""
    import torch
    kw = dict(case)
    n = kw.pop("n")
    p = W.problem_periodic_cube(n, seed=13, prec=prec, **kw)
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, spin_diagonal=True, keep_f64=(prec == "f32")))
    assert h.info["spin_diagonal"] == 1
    stored = tbh.build_hamiltonian(ctx, **tbh.problem_args(p))
    print(f"{name} {prec}: hx bytes spin-diagonal {h.info['hx_bytes']} stored {stored.info['hx_bytes']}",
          flush=True)
    assert h.info["hx_bytes"] < 0.5 * stored.info["hx_bytes"]
    rng = np.random.default_rng(2)
    x, xt = _rand_x(p, rng, True, h.torch_dtype())
    xd = xt.cuda()
    y = tbh.apply_h(h, xd)
    y2 = tbh.apply_h(h, xd)
    torch.cuda.synchronize()
    assert torch.equal(y, y2)
    H = T.hamiltonian(p)
    xr = xt.numpy().astype(np.complex128)
    yr = H @ xr
    yg = y.cpu().numpy().astype(np.complex128)
    row_bound_check(H, xr, yg, yr, prec)
    err = np.linalg.norm(yg - yr) / np.linalg.norm(yr)
    assert err <= (1e-12 if prec == "f64" else 1e-5), err
    if prec == "f32":
        x64 = torch.tensor(x, dtype=torch.complex128).cuda()
        y64 = tbh.apply_h_f64(h, x64).cpu().numpy()
        assert np.linalg.norm(y64 - H @ x) / np.linalg.norm(H @ x) <= 1e-12


def test_spin_diagonal_lanczos_equals_stored(ctx):
    """The fused Lanczos step through the spin-diagonal format on the C2
    recipe at 2^3 cells (FP64): 40 coefficients equal the stored format's to
    1e-10, and the converged values nearest mid-gap are dense eigenvalues."""
    p = W.c2_hardwall_so(0, n=2, m=400)
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec="f64", spin_diagonal=True))
    hs = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec="f64"))
    a1, b1, _ = tbh.lanczos_run(h, 40, p.v0, reorth=False)
    a2, b2, _ = tbh.lanczos_run(hs, 40, p.v0, reorth=False)
    assert np.abs(a1 - a2).max() < 1e-10 and np.abs(b1 - b2).max() < 1e-10
    r = tbh.lanczos_eigs(h, p.sigma, 4, 400, p.v0, reorth=True)
    ev = np.linalg.eigvalsh(T.hamiltonian(p).toarray())
    for e in r["refined"]:
        assert np.abs(ev - e).min() < 1e-9


@pytest.mark.parametrize("bad", [dict(spin=0), dict(spin=1, kfrac=(0.1, 0.0, 0.0))], ids=["no_spin", "kpoint"])
def test_spin_diagonal_rejects_other_models(ctx, bad):
    p = W.problem_periodic_cube(2, seed=3, model=W.MODEL_SP3S, **bad)
    with pytest.raises(tbh.TBHError):
        tbh.build_hamiltonian(ctx, **tbh.problem_args(p, spin_diagonal=True))


def test_handles_destroyed_in_any_order():
    """Contexts, hams, SCF loops and batches may be destroyed in any order
    (a child keeps its parent alive until it is destroyed itself): here the
    context goes first, then the ham, then the loop that uses the ham, and
    the loop still steps between the two."""
    import ctypes as C
    import torch
    lib = tbh.lib()
    p = W.c5_slab(0, nx=2, ny=2, nz=4, n_donors=2)
    ge = p.extra["gap"]
    ctx = tbh.Context(0)
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec="f64"))
    scf = tbh.SCF(h, p.extra["grid"], p.extra["donor_atoms"], p.v0, ge["mid"], ge["cbm"], W.H_GRID_NM,
                  n_cand=32, lanczos_iter=p.dim)
    X = torch.zeros((p.dim, 16), dtype=torch.float32, device="cuda")
    hm = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec="f32", multi_vector=True))
    b = tbh.Batch(ctx, [hm], [X], [torch.empty_like(X)])
    # destroy through the ABI directly, parents first
    assert lib.tbh_ctx_destroy(ctx.h) == tbh.TBH_OK
    ctx.h = None
    assert lib.tbh_ham_destroy(hm.h) == tbh.TBH_OK
    hm.h = None
    b.apply()
    assert lib.tbh_ham_destroy(h.h) == tbh.TBH_OK
    h.h = None
    r = scf.step()
    assert np.isfinite(r["residual"])
    scf.close()
    b.close()
