"""The trained start-potential surrogate against the plain method on
donor layouts it was not trained on (seeds outside the training range), and
the fallback rule, forced from the host.

The network is the committed one, trained with the library's own kernels
on converged plain-method potentials of the study slab (3x3x8 cells, 9
donors, 4 K).  Bars: the learned start's max-norm error against the
converged potential is at most a tenth of the zero start's, the loop from it
converges in fewer steps, and both starts reach the same fixed point
(within 1e-3 eV).  A start far from any solution (-60 eV everywhere) trips
the "first residual > 10x the zero start's" rule and the loop still
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


def test_learned_start_beats_zero_start(study):
    start = study.surrogate(WEIGHTS)
    for seed in (2000, 2001):
        assert seed not in start.train_seeds
        p = W.study_slab(seed)
        zero = study.run(seed, None, 400)
        assert zero["converged"]
        U0 = start(study.donor_map(p))
        e_learned = float((U0 - zero["U"]).abs().max())
        e_zero = float(zero["U"].abs().max())
        learned = study.run(seed, U0, 400, zero["residuals"][0], fallback=True)
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
    bad = torch.full((nz, ny, nx), -60.0, dtype=torch.float64, device="cuda")
    r = study.run(seed, bad, 400, zero_first, fallback=True)
    assert r["fell_back"]
    assert r["converged"]
