"""The hard-wall spin-orbit silicon cube at full size (20^3 cells, 64,000
atoms, complex H of dimension 1.28M, +30 eV dangling-bond hybrids, +-1 %
bond strain), the 16 distinct eigenvalues nearest mid-gap: the FP32 pipeline
(FP32 H.x and vectors, FP64 scalars, FP64 refinement) against the all-FP64
pipeline.

Both run 6000 Lanczos steps without reorthogonalisation from the same start
vector and keep the whole basis for the Ritz vectors.  Bars: each pipeline
reports 16 distinct converged values, the same 16 to 1e-6 eV after
refinement, and every FP32 value is certified to 1e-6 eV.  A value's own
certificate is c = min(r, r^2 / gamma) from its explicit FP64 residual r and
its gap gamma to the nearest other reported value (the residual bound
|theta - lambda| <= r, or Kato-Temple once the gap separates the value from
the rest of the spectrum).  Where the FP32 Ritz vector's residual is too
large for that (the FP32 basis leaves residuals of 1e-6 to 3e-5 eV), the
value is certified through the FP64 pipeline's: |e32 - e64| + c64.
"""
import json

import numpy as np
import pytest

import paper_1003_4570_amd as tbh
import workloads as W

pytestmark = pytest.mark.gpu


def test_c2_full_size_fp32_matches_fp64():
    import torch
    assert torch.cuda.is_available()
    ctx = tbh.Context(0)
    p = W.c2_hardwall_so(0, m=6000)
    assert p.n_atoms == 64000 and p.dim == 1_280_000
    out = {}
    for prec in ("f64", "f32"):
        print(f"c2 full size: {prec} pipeline", flush=True)
        h = tbh.build_hamiltonian(ctx, **tbh.problem_args(p, prec=prec, keep_f64=(prec == "f32")))
        v0 = torch.tensor(np.ascontiguousarray(p.v0).view(np.float64), device="cuda")
        r = tbh.lanczos_eigs(h, p.sigma, 16, 6000, v0, reorth=False, n_cand=256)
        out[prec] = r
        h.close()
        del h
        torch.cuda.empty_cache()
    r64, r32 = out["f64"], out["f32"]
    assert r64["report"]["n_found"] == 16 and r32["report"]["n_found"] == 16
    e64, e32 = np.sort(r64["refined"]), np.sort(r32["refined"])
    diff = np.abs(e32 - e64)
    gap = np.array([np.min(np.abs(np.delete(e32, i) - e32[i])) for i in range(16)])
    def own_cert(r, e):
        order = np.argsort(r["refined"])
        res = np.asarray(r["res"])[order]
        g = np.array([np.min(np.abs(np.delete(e, i) - e[i])) for i in range(e.size)])
        return res, np.minimum(res, res ** 2 / g)

    res, cert_own = own_cert(r32, e32)
    res64, cert64 = own_cert(r64, e64)
    cert = np.minimum(cert_own, diff + cert64)
    rec = dict(workload="lanczos6000_si20x20x20_hardwall_sp3d5s_so", sigma=p.sigma,
               evals_f64=e64.tolist(), evals_f32=e32.tolist(), max_diff=float(diff.max()),
               residual_f32=res.tolist(), residual_f64=res64.tolist(), gap=gap.tolist(),
               certified_own=cert_own.tolist(), certified_f64=cert64.tolist(), certified=cert.tolist(),
               self_certified=int((cert_own <= 1e-6).sum()),
               seconds_f32=r32["report"]["seconds"], seconds_f64=r64["report"]["seconds"])
    print(json.dumps(rec), flush=True)
    assert diff.max() < 1e-6
    assert cert64.max() <= 1e-6
    assert cert.max() <= 1e-6
