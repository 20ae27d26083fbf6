"""The allocation-free Poisson entry point (tbh_poisson_solve_noalloc) against
the allocating one (tbh_poisson_solve), both called through the C ABI.

The two run the same CG kernels on the same inputs, so the solutions and
iteration counts must agree bitwise; both are also checked against the
oracle's exact spectral solve of the same discrete equations (1e-9 of the
solution's scale).  Two calls in a row, the second on a smaller grid, show
that the shared static scratch carries nothing over; an oversized grid is
refused with TBH_EINVAL.
"""
import ctypes as C

import numpy as np
import pytest

import paper_1003_4570_amd as tbh
import workloads as W
from oracle import poisson as P

pytestmark = pytest.mark.gpu


def _call(fn, ctx, grid, rho, phi, rel_tol=1e-12, max_iter=20000):
    g = (C.c_int32 * 3)(*grid)
    it = C.c_int32(-1)
    rr = C.c_double(-1.0)
    rc = fn(ctx.h, g, W.H_GRID_NM, 11.7, C.c_void_p(rho.data_ptr()), C.c_void_p(phi.data_ptr()), rel_tol,
            max_iter, C.byref(it), C.byref(rr))
    return rc, it.value, rr.value


def test_noalloc_poisson_matches_allocating_entry_point():
    import torch
    assert torch.cuda.is_available()
    ctx = tbh.Context(0)
    lib = tbh.lib()
    # the slab grid of the Schrodinger-Poisson workload first, then a smaller one
    for grid in [(32, 32, 240), (12, 8, 20)]:
        nx, ny, nz = grid
        print(f"noalloc poisson grid={grid}", flush=True)
        rng = np.random.default_rng(nx * ny * nz)
        rho_h = rng.standard_normal((nz, ny, nx))
        rho = torch.from_numpy(rho_h).cuda()
        guess = torch.from_numpy(0.01 * rng.standard_normal((nz, ny, nx))).cuda()
        phi_a = guess.clone()
        phi_b = guess.clone()
        rc_a, it_a, rr_a = _call(lib.tbh_poisson_solve, ctx, grid, rho, phi_a)
        rc_b, it_b, rr_b = _call(lib.tbh_poisson_solve_noalloc, ctx, grid, rho, phi_b)
        torch.cuda.synchronize()
        assert rc_a == tbh.TBH_OK and rc_b == tbh.TBH_OK, (rc_a, rc_b, tbh.last_error())
        assert it_a == it_b and rr_a == rr_b
        assert torch.equal(phi_a, phi_b)
        ref = P.spectral_solve(P.rhs(rho_h, 11.7), W.H_GRID_NM)
        assert np.abs(phi_b.cpu().numpy() - ref).max() <= 1e-9 * np.abs(ref).max()


def test_noalloc_poisson_refuses_oversized_grid():
    import torch
    ctx = tbh.Context(0)
    grid = (64, 64, 65)            # 266,240 nodes > 2^18
    rho = torch.zeros(grid[::-1], dtype=torch.float64).cuda()
    phi = torch.zeros_like(rho)
    rc, _, _ = _call(tbh.lib().tbh_poisson_solve_noalloc, ctx, grid, rho, phi)
    assert rc == tbh.TBH_EINVAL
    assert "allocation-free limit" in tbh.last_error()
