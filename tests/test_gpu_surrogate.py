"""The trained start-potential surrogate against the plain method on donor
layouts it was not trained on (seeds outside the training range), the start
built by the library (tbh_scf_set_start) against the same arithmetic written
out with torch, and the fallback rule.

The network is the committed one, trained with the library's own kernels
on converged plain-method potentials of the study slab (3x3x8 cells, 9
donors, 4 K).  Bars: the device start equals the torch assembly to 1e-5 eV;
the learned start's max-norm error against the converged potential is at
most a tenth of the zero start's, the loop from it converges in fewer steps,
and both starts reach the same fixed point (within 1e-3 eV).  A start far
from any solution (-60 eV below the bare-donor potential) trips the "first
residual > 10x the zero start's" rule inside the library and the loop still
converges from zero.
"""
import os

import numpy as np
import pytest

import paper_1003_4570_amd as tbh
from paper_1003_4570_amd import surrogate as S
import workloads as W

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(tbh.__file__), "data", "surrogate_study_slab.npz")


@pytest.fixture(scope="module")
def study():
    import torch
    assert torch.cuda.is_available()
    return S.Study()


def test_bare_potential_is_poisson_of_donors(study):
    """The bare-donor input map: a single donor's potential is negative,
    deepest at the donor's node, and linear in the donor count."""
    import torch
    nx, ny, nz = study.grid
    d = np.zeros((nz, ny, nx), np.float32)
    d[nz // 2, 3, 5] = 1.0
    u1 = study.bare_potential(d)
    u2 = study.bare_potential(2 * d)
    assert float(u1.max()) <= 0.0
    assert int(torch.argmin(u1)) == (nz // 2 * ny + 3) * nx + 5
    assert torch.allclose(u2, 2 * u1, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("kind", ["learned", "mean"])
def test_device_start_equals_torch_assembly(study, kind):
    """U0 = U_bare + mean (+ scale * the average over the four point
    operations of op^-1 net(op x)) built by tbh_scf_set_start equals the
    same formula evaluated here with torch index operations and the
    network's forward entry point."""
    import torch
    start = study.surrogate(WEIGHTS)
    seed = 2003
    p = W.study_slab(seed)
    dmap = study.donor_map(p)
    rec = study.run(seed, start, 1, mean_only=(kind == "mean"))
    U0 = rec["U0"]
    ub = study.bare_potential(dmap)
    want = ub + start.Tbar.double()
    if kind == "learned":
        x = study.inputs(dmap, start.feat_scale)
        y = sum(inv(start.net.forward(op(x).contiguous())) for op, inv in S.point_ops()) / 4.0
        want = want + start.scale * y.double()
    d = float((U0 - want).abs().max())
    print(f"{kind}: max |U0_device - U0_torch| = {d:.2e} eV", flush=True)
    assert d < 1e-5


def test_learned_start_beats_zero_start(study):
    start = study.surrogate(WEIGHTS)
    for seed in (2000, 2001):
        assert seed not in start.train_seeds
        zero = study.run(seed, None, 400)
        assert zero["converged"]
        learned = study.run(seed, start, 400, 10 * zero["residuals"][0])
        e_learned = float((learned["U0"] - zero["U"]).abs().max())
        e_zero = float(zero["U"].abs().max())
        print(f"seed {seed}: err0 zero {e_zero:.3f} learned {e_learned:.4f} eV; steps zero "
              f"{zero['iterations']} learned {learned['iterations']}", flush=True)
        assert e_learned < 0.1 * e_zero
        assert learned["converged"] and not learned["fell_back"]
        assert learned["iterations"] < zero["iterations"]
        assert float((learned["U"] - zero["U"]).abs().max()) < 1e-3


def test_fallback_on_far_start(study):
    import torch
    seed = 2002
    nx, ny, nz = study.grid
    zero_first = study.run(seed, None, 1)["residuals"][0]
    bad = torch.full((nz, ny, nx), -60.0, dtype=torch.float32, device="cuda")
    r = study.run(seed, None, 400, 10 * zero_first, fixed_start=bad)
    assert r["fell_back"]
    assert r["converged"]
