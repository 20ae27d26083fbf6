"""Find synthetic parameter sets with a bulk band gap (writes workloads/gap_table.json).

TEST INFRASTRUCTURE ONLY: a committed script that calls only the oracle.

The paper's structures are semiconductors described by bulk-calibrated
tight-binding parameters (Sec. I); the published Si/Ge parameter tables are
not part of the paper, so the workloads draw synthetic parameters.  A random
set is usable for "states near the gap" only if its bulk bands have a gap.
This script draws parameter seeds 0, 1, 2, ... (the same draw the workloads
make) and accepts the first whose bulk diamond bands, sampled on a 16^3
grid of the Brillouin zone plus the Gamma, X and L points, leave a gap of at
least 0.5 eV above the valence bands (4 bands per spin; 8 with spin-orbit).

    python -m oracle.gap_search
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import tb as T  # noqa: E402


def kpoints(n=16):
    """Cartesian k (units of 1/(a/4)) on an n^3 grid of the fcc Brillouin zone
    plus Gamma, X and L."""
    g = np.pi / 2.0                           # 2 pi / a with a = 4
    b = g * np.array([[-1, 1, 1], [1, -1, 1], [1, 1, -1]], dtype=float)
    f = (np.arange(n) + 0.5) / n
    fa, fb, fc = np.meshgrid(f, f, f, indexing="ij")
    ks = fa.ravel()[:, None] * b[0] + fb.ravel()[:, None] * b[1] + fc.ravel()[:, None] * b[2]
    special = np.array([[0, 0, 0], [g, 0, 0], [g / 2, g / 2, g / 2]])
    return np.vstack([special, ks])


def band_edges(par, ks):
    model, spin = par["model"], par["spin"]
    nval = 4 * (2 if spin else 1)
    vbm, cbm = -np.inf, np.inf
    for k in ks:
        e = np.linalg.eigvalsh(T.bulk_hk(model, spin, par["onsite"][0], par["sk"][0][0],
                                         par["so_delta"][0], k))
        vbm = max(vbm, e[nval - 1])
        cbm = min(cbm, e[nval])
    return vbm, cbm


def search(model, spin, min_gap=0.5, max_seed=5000, n=16):
    ks_coarse = kpoints(6)
    ks = kpoints(n)
    for seed in range(max_seed):
        par = W.draw_params(np.random.default_rng(seed), model, spin, 1)
        v, c = band_edges(par, ks_coarse)
        if c - v < min_gap:
            continue
        v, c = band_edges(par, ks)
        if c - v >= min_gap:
            return dict(seed=seed, vbm=float(v), cbm=float(c), mid=float(0.5 * (v + c)),
                        gap=float(c - v), model=model, spin=spin, grid=n)
    raise RuntimeError("no gap-accepted parameter seed found")


def main():
    out = {}
    for model, spin in ((W.MODEL_SP3D5S, 0), (W.MODEL_SP3D5S, 1), (W.MODEL_SP3S, 0), (W.MODEL_SP3S, 1)):
        e = search(model, spin)
        out[f"model{model}_spin{spin}"] = e
        print(e, flush=True)
    path = os.path.join(ROOT, "workloads", "gap_table.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
