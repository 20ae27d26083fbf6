"""GPU parity of the Poisson solver and the Schrodinger-Poisson loop.

* FP64 CG Poisson vs the oracle's spectral solve of the same discrete
  equations (relative 1e-9 at CG tolerance 1e-12), several grid shapes;
* SCF on a small delta-doped slab (C5 recipe: sp3d5s*, hard-wall z with
  +30 eV passivation, donors in the mid plane, 4 K) with the full Krylov
  space (every eigenpair) against the oracle's dense SCF: the potential
  iterate by iterate to 1e-8 eV, Fermi levels and residuals alike.
"""
import numpy as np
import pytest

import paper_1003_4570_amd as tbh
import workloads as W
from oracle import poisson as P
from oracle import scf as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return tbh.Context(0)


@pytest.mark.parametrize("shape", [(24, 8, 8), (240, 32, 32), (7, 5, 3)])
def test_poisson_cg_vs_spectral(ctx, shape):
    import torch
    rng = np.random.default_rng(sum(shape))
    rho = rng.standard_normal(shape)
    h, eps = W.H_GRID_NM, 11.7
    phi, it, rr = tbh.poisson_solve(ctx, shape[::-1], h, eps, torch.tensor(rho).cuda(), rel_tol=1e-12)
    ref = P.spectral_solve(P.rhs(rho, eps), h)
    print(shape, "cg iters", it, "rel", rr, flush=True)
    assert rr <= 1e-12
    assert np.abs(phi.cpu().numpy() - ref).max() <= 1e-9 * np.abs(ref).max()


def test_poisson_nonconvergence_reported(ctx):
    import torch
    rho = torch.ones((40, 16, 16), dtype=torch.float64, device="cuda")
    phi, it, rr = tbh.poisson_solve(ctx, (16, 16, 40), W.H_GRID_NM, 11.7, rho, rel_tol=1e-14, max_iter=3)
    assert it == 3 and rr > 1e-14


def _slab():
    p = W.c5_slab(0, nx=2, ny=2, nz=4, n_donors=3)
    rng = np.random.default_rng(7)
    grid = p.extra["grid"]
    U0 = rng.uniform(-0.05, 0.05, size=grid[::-1])   # breaks the lattice symmetry
    return p, grid, U0


@pytest.mark.parametrize("fixed", [False, True])
def test_scf_iterates_match_oracle(ctx, fixed):
    import torch
    p, grid, U0 = _slab()
    ge = p.extra["gap"]
    donors = p.extra["donor_atoms"]
    nit = 4
    ef = ge["cbm"] - 0.3 if fixed else None
    ro = S.scf(p, donors, grid, U0, ge["mid"], alpha=0.1, tol=1e-12, max_iter=nit, Ef_fixed=ef)
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec="f64"))
    dim = p.dim
    scf = tbh.SCF(h, grid, donors, p.v0, ge["mid"], ge["cbm"], W.H_GRID_NM, mix_alpha=0.1,
                  tol_eV=1e-12, n_cand=dim, lanczos_iter=dim, res_tol=1e-6, fermi_fixed=ef)
    scf.set_potential(torch.tensor(U0).cuda())
    for t in range(nit):
        Ug = scf.potential().cpu().numpy()
        err = np.abs(Ug - ro["iterates"][t]).max()
        r = scf.step()
        print(f"iter {t} |dU|={err:.3e} res gpu {r['residual']:.6e} oracle {ro['residuals'][t]:.6e} "
              f"Ef {r['fermi']:.9f} / {ro['Ef'][t]:.9f} states {r['n_cb']} conv {r['n_conv']}", flush=True)
        assert err < 1e-8
        assert r["n_conv"] == dim
        assert abs(r["residual"] - ro["residuals"][t]) < 1e-8
        assert abs(r["fermi"] - ro["Ef"][t]) < 1e-8
        assert abs(r["electrons"] - (len(donors) if not fixed else r["electrons"])) < 1e-8


def _dense_step(p, grid, U, T_K=4.0):
    """One step of the oracle's loop body at potential U (dense eigenpairs,
    Fermi level by neutrality, CG Poisson): its output potential."""
    from oracle import tb as T
    blk = T.build_blocks(p)
    H0 = T.csr_hamiltonian(blk).toarray()
    nodes = S.node_index(p.pos_q, grid)
    nx, ny, nz = grid
    nd = np.zeros(nx * ny * nz)
    np.add.at(nd, nodes[p.extra["donor_atoms"]], 1.0)
    o = S.loop_body(H0, blk["n_o"], nodes, nd, U, grid, p.extra["gap"]["mid"], float(len(p.extra["donor_atoms"])),
                    S.KB_EV * T_K, W.H_GRID_NM, 11.7, None, 1e-12)
    return o["U_out"]


@pytest.mark.parametrize("mode", [0, 1], ids=["lanczos_cgs2", "filtered_block"])
def test_scf_production_setting_is_an_oracle_fixed_point(ctx, mode):
    """The study slab (3x3x8 cells, 9 donors, 4 K) in the production setting:
    FP32 H with its FP64 copy, linear mixing 0.05 to 1e-4 eV, and either 64
    candidates of 800 CGS2 Lanczos steps or the filtered block solver (block
    64).  The converged potential is a fixed point of one dense FP64 oracle
    step: |U_out - U| < 1e-4 eV at every node."""
    import torch
    p = W.study_slab(1003)
    ge = p.extra["gap"]
    grid = p.extra["grid"]
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec="f32", keep_f64=True, multi_vector=(mode == 1)))
    kw = dict(mix_alpha=0.05, tol_eV=1e-4, res_tol=1e-4, T_K=4.0)
    if mode == 0:
        kw.update(n_cand=64, lanczos_iter=800)
    else:
        kw.update(eig_mode=1, block=64, filter_degree=20, filter_degree_cold=80, filter_max_iter=60, k_states=40,
                  e_vbm=ge["vbm"])
    scf = tbh.SCF(h, grid, p.extra["donor_atoms"], p.v0, ge["mid"], ge["cbm"], W.H_GRID_NM, **kw)
    r = scf.run(400)
    print(f"mode {mode}: steps {r['iterations']} residual {r['residual']:.2e} seconds {r['seconds']:.2f}", flush=True)
    assert r["converged"]
    U = scf.potential().cpu().numpy()
    U_out = _dense_step(p, grid, U)
    d = np.abs(U_out - U).max()
    print(f"dense oracle step from the GPU's U: max |U_out - U| = {d:.2e} eV", flush=True)
    assert d < 1e-4


def test_filtered_eigs_lowest_conduction_states(ctx):
    """Filtered subspace iteration on (H - s)^2 (s three quarters into the
    bulk gap) on a 3x3x20-cell slab: the 40 lowest conduction states equal
    the reference spectrum's to 1e-6 eV (degenerate copies counted), with FP64
    residuals of the returned unit vectors <= 1e-4 eV."""
    from scipy.sparse.linalg import eigsh
    from oracle import tb as T
    p = W.c5_slab(1000, nx=3, ny=3, nz=20, n_donors=9)
    ge = p.extra["gap"]
    H = T.hamiltonian(p)
    # reference: shift-invert Lanczos (ARPACK) on the FP64 CSR H below the band edge
    ev = np.sort(eigsh(H, k=80, sigma=ge["cbm"] - 0.5, which="LM", return_eigenvectors=False))
    want = ev[ev > ge["mid"]][:40]
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec="f32", keep_f64=True, multi_vector=True))
    s = ge["vbm"] + 0.75 * (ge["cbm"] - ge["vbm"])
    r = tbh.filtered_eigs(h, s, 40, 64, degree=40, degree_cold=80, max_iter=60, want_vectors=True)
    print("report", r["report"], flush=True)
    assert r["report"]["n_found"] == 40
    assert np.abs(r["evals"] - want).max() < 1e-6
    Y = r["vectors"].cpu().numpy()
    R = (H @ Y.T) - Y.T * r["evals"][None, :]
    assert np.linalg.norm(R, axis=0).max() < 1e-4
    assert np.abs(Y @ Y.T - np.eye(40)).max() < 1e-5


@pytest.mark.parametrize("fixed", [False, True])
def test_newton_iterates_match_oracle(ctx, fixed):
    """Newton-Raphson updates (Jacobian from the 64 lowest filled-class
    states, occupations smeared at 10 meV inside it, Anderson depth 4) on the
    small slab with the full Krylov space, against the oracle's dense Newton
    loop from the same start: the potential iterate by iterate to 1e-8 eV."""
    import torch
    from oracle import newton as NW
    p, grid, U0 = _slab()
    ge = p.extra["gap"]
    donors = p.extra["donor_atoms"]
    nit = 5
    ef = ge["cbm"] - 0.3 if fixed else None
    ro = NW.scf_newton(p, donors, grid, U0, ge["mid"], tol=1e-12, max_iter=nit, Ef_fixed=ef, n_states=64,
                       kT_J=0.01, depth=4)
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec="f64"))
    dim = p.dim
    scf = tbh.SCF(h, grid, donors, p.v0, ge["mid"], ge["cbm"], W.H_GRID_NM, tol_eV=1e-12, n_cand=dim,
                  lanczos_iter=dim, res_tol=1e-6, fermi_fixed=ef, update_mode=1, newton_states=64, newton_kT=0.01,
                  anderson_depth=4, newton_cg_tol=1e-13)
    scf.set_potential(torch.tensor(U0).cuda())
    for t in range(nit):
        Ug = scf.potential().cpu().numpy()
        err = np.abs(Ug - ro["iterates"][t]).max()
        r = scf.step()
        print(f"iter {t} |dU|={err:.3e} res gpu {r['residual']:.6e} oracle {ro['residuals'][t]:.6e} "
              f"pairs {r['newton_pairs']} cg {r['newton_cg_iters']}", flush=True)
        assert err < 1e-8
        assert abs(r["residual"] - ro["residuals"][t]) < 1e-8


@pytest.mark.parametrize("mode", [0, 1], ids=["lanczos_cgs2", "filtered_block"])
def test_newton_production_setting_is_an_oracle_fixed_point(ctx, mode):
    """The study slab in the production setting with the Newton-Raphson
    update: converges in at most 40 steps (linear mixing needs about 190),
    and the converged potential is a fixed point of one dense FP64 oracle
    step (|U_out - U| < 1e-4 eV at every node)."""
    p = W.study_slab(1003)
    ge = p.extra["gap"]
    grid = p.extra["grid"]
    h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec="f32", keep_f64=True, multi_vector=(mode == 1)))
    kw = dict(mix_alpha=0.05, tol_eV=1e-4, res_tol=1e-4, T_K=4.0, update_mode=1)
    if mode == 0:
        kw.update(n_cand=64, lanczos_iter=800)
    else:
        kw.update(eig_mode=1, block=64, filter_degree=20, filter_degree_cold=80, filter_max_iter=60, k_states=40,
                  e_vbm=ge["vbm"])
    scf = tbh.SCF(h, grid, p.extra["donor_atoms"], p.v0, ge["mid"], ge["cbm"], W.H_GRID_NM, **kw)
    r = scf.run(100)
    print(f"newton mode {mode}: steps {r['iterations']} residual {r['residual']:.2e} seconds {r['seconds']:.2f}",
          flush=True)
    assert r["converged"] and r["iterations"] <= 40
    U = scf.potential().cpu().numpy()
    d = np.abs(_dense_step(p, grid, U) - U).max()
    print(f"dense oracle step from the GPU's U: max |U_out - U| = {d:.2e} eV", flush=True)
    assert d < 1e-4
