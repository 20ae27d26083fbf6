"""Benchmark: H.x throughput inside the Lanczos iteration on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one pass of the measured path over the million-atom workload: 500
Lanczos iterations (the paper's benchmark unit, Sec. II-B, Figs. 2-3) on a
periodic random Si(0.7)Ge(0.3) alloy of 51^3 conventional cells (1,061,208
atoms), sp3d5s* without spin (10 orbitals, real symmetric H of dimension
10,612,080), FP32 H.x and Lanczos vectors with FP64 inner products, no
reorthogonalisation.  Inputs (H, start vector) are resident in HBM before the
timed region.

value = algorithmic bytes of the fused Lanczos H.x moved per second over the
whole timed job (packed H + neighbour table + x once + y once + x_prev once,
per iteration, times the iterations), the Lanczos vector updates and
reductions included in the time.

roofline: the fused Lanczos H.x kernel's algorithmic bytes per launch over
its average launch duration, timed with HIP events on the stream it runs on;
traffic: HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE counter
runs (profiles/hx_c3_counters.txt), reported only while the kernel source is
the one the counters were taken on.

cpu_baseline: the CPU oracle (scipy CSR, FP64) running the same recurrence on
a bounded sample of the same workload (a 16^3-cell alloy block), converted to
the same bytes-per-atom unit.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ITERS_PER_STEP = 500


def _kernel_hash():
    h = hashlib.sha256()
    for f in ("hx.hip", "tbh_internal.h"):
        with open(os.path.join(ROOT, "paper_1003_4570_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(bytes_alg):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "hx_c3_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_hash") != _kernel_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(seconds_budget=20.0):
    """The oracle's FP64 CSR Lanczos recurrence (no reorthogonalisation) on a
    16^3-cell block of the same alloy recipe, timed on the host."""
    from threadpoolctl import threadpool_limits
    import workloads as W
    from oracle import lanczos as L
    from oracle import tb as T
    p = W.c3_alloy(0, n=16, m=ITERS_PER_STEP)
    H = T.hamiltonian(p)
    per_atom = 4 * 400 + 40 + 16 + 40 + 40      # same bytes/atom as the GPU format (FP32)
    it = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        # recurrence chunks until the time budget is used
        while True:
            L.lanczos(lambda x: H @ x, p.v0, 20, reorth=False)
            it += 20
            if time.perf_counter() - t0 > seconds_budget or it >= 2000:
                break
        dt = time.perf_counter() - t0
    gbs = per_atom * p.n_atoms * it / dt / 1e9
    return dict(value=gbs, unit="GB/s", cores=1, kind="oracle",
                sample=f"scipy CSR FP64 Lanczos recurrence, {it} iterations on a 16^3-cell "
                       f"Si0.7Ge0.3 block ({p.n_atoms} atoms, sp3d5s*), bytes counted in the "
                       f"GPU's FP32 per-atom format ({per_atom} B/atom/H.x)")


def calibrate_copy():
    """A plain device copy of known size, for scaling FETCH_SIZE/WRITE_SIZE."""
    import torch
    n = 1 << 28  # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": n * 4, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported (single-GPU build)",
              file=sys.stderr)
        sys.exit(2)
    if a.calibrate_copy:
        calibrate_copy()
        return

    import torch
    import paper_1003_4570_amd as tbh
    import workloads as W

    print("bench: building the 51^3-cell alloy Hamiltonian", file=sys.stderr, flush=True)
    prob = W.c3_alloy(0)
    ctx = tbh.Context(0)
    ham = tbh.build_hamiltonian(ctx, **tbh.problem_args(prob))
    v0 = torch.tensor(prob.v0, dtype=torch.float64, device="cuda")
    # the fused step kernel also reads x_prev (the beta_j v_{j-1} term)
    hx_bytes = ham.info["hx_bytes"] + ham.info["dim"] * 4
    torch.cuda.synchronize()

    for _ in range(a.warmup):
        tbh.lanczos_run(ham, ITERS_PER_STEP, v0, reorth=False)
    torch.cuda.synchronize()
    print("bench: timed region", file=sys.stderr, flush=True)
    hx_s = 0.0
    steps_done = 0
    t0 = time.perf_counter()
    for _ in range(a.steps):
        _, _, rep = tbh.lanczos_run(ham, ITERS_PER_STEP, v0, reorth=False, time_hx=True)
        hx_s += rep["hx_seconds"]
        steps_done += rep["steps"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_hx = steps_done
    value = hx_bytes * n_hx / dt / 1e9
    hx_avg = hx_s / n_hx
    achieved = hx_bytes / hx_avg / 1e9
    traffic = _traffic(hx_bytes)
    out = {
        "metric": "H.x GB/s in Lanczos (fraction of HBM peak)",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(dt / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lanczos500_si0.7ge0.3_51x51x51_sp3d5s_fp32",
                   "atoms": ham.info["n_atoms"], "dim": ham.info["dim"],
                   "lanczos_iterations_per_step": ITERS_PER_STEP, "reorth": "none",
                   "hx_bytes_per_launch": hx_bytes},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "hx_kernel<float,real,10,10,diag,lanczos>",
                     "avg_launch_ms": round(hx_avg * 1e3, 4)},
    }
    if not a.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
