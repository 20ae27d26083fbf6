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
a bounded sample of the same workload (a 16^3-cell alloy block), one process
per host core, converted to the same bytes-per-atom unit.

scf_learned_vs_plain: the metric's second half, measured in the run: SCF
time-to-converge (1e-4 eV) on the 8x8x60-cell delta-doped slab from the zero
start and from the learned start, on held-out donor layouts.
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
    # the kernel, its layout, and the builder (which fixes the atom order)
    for f in ("hx.hip", "tbh_internal.h", "builder.cpp"):
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


C3_METHOD_BYTES_PER_ATOM = 4 * 400 + 40 + 16 + 40 + 40 + 40   # bonds, diagonal on-site, nbr, x, y, x_prev


def _oracle_worker(args):
    """One process: the oracle's FP64 CSR Lanczos recurrence on the sample
    block until the time budget is used; returns (iterations, seconds)."""
    seconds_budget, seed = args
    from threadpoolctl import threadpool_limits
    import workloads as W
    from oracle import lanczos as L
    from oracle import tb as T
    p = W.c3_alloy(seed, n=16, m=ITERS_PER_STEP)
    H = T.hamiltonian(p)
    it = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while True:
            L.lanczos(lambda x: H @ x, p.v0, 20, reorth=False)
            it += 20
            if time.perf_counter() - t0 > seconds_budget or it >= 4000:
                break
        dt = time.perf_counter() - t0
    return it, dt, p.n_atoms


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds_budget=20.0):
    """The oracle's FP64 CSR Lanczos recurrence (no reorthogonalisation) on a
    16^3-cell block of the same alloy recipe, timed on the host: one process
    per available core (scipy's CSR product is single-threaded, so the
    machine's throughput is that of independent recurrences), and one
    process alone."""
    import multiprocessing as mp
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    ncores = max(1, min(ncores, 16))
    ctx = mp.get_context("spawn")
    with ctx.Pool(ncores) as pool:
        runs = pool.map(_oracle_worker, [(seconds_budget, s) for s in range(ncores)])
    with ctx.Pool(1) as pool:
        single = pool.map(_oracle_worker, [(seconds_budget, 0)])[0]
    per_atom = C3_METHOD_BYTES_PER_ATOM
    total = sum(per_atom * n * it / dt for it, dt, n in runs) / 1e9
    one = per_atom * single[2] * single[0] / single[1] / 1e9
    return dict(value=round(total, 3), unit="GB/s", cores=ncores, kind="oracle",
                single_core_value=round(one, 3), cpu_model=_cpu_model(),
                sample=f"scipy CSR FP64 Lanczos recurrence (no reorthogonalisation) on a 16^3-cell Si0.7Ge0.3 "
                       f"block ({runs[0][2]} atoms, sp3d5s*), one independent process per core "
                       f"({ncores} processes, {sum(r[0] for r in runs)} iterations in about {seconds_budget:.0f} s "
                       f"each; scipy's CSR product uses one thread), bytes counted with the method's "
                       f"{per_atom} B/atom per fused step")


def scf_leg(seeds, max_iter=600):
    """SCF time-to-converge on the 8x8x60-cell delta-doped slab (30,720
    atoms, 64 donors, 4 K, linear mixing 0.05 to 1e-4 eV): the zero start
    against the learned start (the committed network, built on the device by
    tbh_scf_set_start, its time included), on held-out donor layouts; and, as
    context, the zero start with the Newton-Raphson update."""
    import paper_1003_4570_amd as tbh
    from paper_1003_4570_amd import surrogate as S
    weights = os.path.join(ROOT, "paper_1003_4570_amd", "data", "surrogate_c5.npz")
    if not os.path.exists(weights):
        return None
    st = S.Study(geometry="c5")
    start = st.surrogate(weights)
    recs = []
    for sd in seeds:
        print(f"bench: SCF layout {sd}, zero start", file=sys.stderr, flush=True)
        zero = st.run(sd, None, max_iter)
        print(f"bench: SCF layout {sd}, learned start", file=sys.stderr, flush=True)
        learned = st.run(sd, start, max_iter, 10.0 * zero["residuals"][0])
        print(f"bench: SCF layout {sd}, zero start, Newton-Raphson update", file=sys.stderr, flush=True)
        newton = st.run(sd, None, max_iter, update_mode=1)
        recs.append(dict(seed=sd, zero_iterations=zero["iterations"], zero_seconds=round(zero["seconds"], 3),
                         newton_zero_iterations=newton["iterations"], newton_zero_seconds=round(newton["seconds"], 3),
                         newton_zero_converged=newton["converged"],
                         zero_converged=zero["converged"], learned_iterations=learned["iterations"],
                         learned_seconds=round(learned["seconds"], 3),
                         learned_start_seconds=round(learned["start_seconds"], 4),
                         learned_converged=learned["converged"], fell_back=learned["fell_back"],
                         fixed_point_diff=float((learned["U"] - zero["U"]).abs().max())))
    zs = float(np.median([r["zero_seconds"] for r in recs]))
    ls = float(np.median([r["learned_seconds"] for r in recs]))
    zi = float(np.median([r["zero_iterations"] for r in recs]))
    li = float(np.median([r["learned_iterations"] for r in recs]))
    return dict(workload="scf_c5_slab8x8x60_sp3d5s_64donors_4K", measured="in this run",
                held_out_seeds=list(seeds), zero_seconds=zs, learned_seconds=ls, zero_iterations=zi,
                learned_iterations=li, speedup_time=round(zs / ls, 3), speedup_iterations=round(zi / li, 3),
                tolerance_eV=1e-4,
                newton_zero_seconds=float(np.median([r["newton_zero_seconds"] for r in recs])),
                newton_zero_iterations=float(np.median([r["newton_zero_iterations"] for r in recs])),
                records=recs)


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


def bench_c2(a):
    """FP32 H.x / FP32 vectors with FP64 scalars against the all-FP64
    pipeline on the 20^3-cell hard-wall spin-orbit cube (64,000 atoms,
    complex H of dimension 1.28M): 16 distinct eigenvalues nearest mid-gap.
    Interior values need thousands of steps; full reorthogonalisation costs
    O(m^2 dim) and converged 2 of them in 3000 steps (37 s, measured), so the
    run keeps the whole basis in HBM (m * 10 MB in FP32, 20 MB in FP64) and
    does not reorthogonalise: ghost copies are merged by value and every
    reported value is certified by its explicit FP64 residual."""
    import torch
    import paper_1003_4570_amd as tbh
    import workloads as W
    m = a.c2_m
    prob = W.c2_hardwall_so(0, m=m)
    ctx = tbh.Context(0)
    out = {"metric": "eigenvalue error FP32 pipeline vs FP64 (eV)", "unit": "eV", "n_gpus": 1,
           "higher_is_better": False, "data": "synthetic", "dtype": "f32",
           "config": {"workload": f"lanczos{m}_si20x20x20_hardwall_sp3d5s_so", "atoms": prob.n_atoms,
                      "k": prob.k, "sigma_eV": prob.sigma, "reorth": "none", "n_cand": a.c2_cand}}
    res = {}
    for prec in ("f64", "f32"):
        print(f"bench c2: build {prec}", file=sys.stderr, flush=True)
        ham = tbh.build_hamiltonian(ctx, **tbh.problem_args(prob, prec=prec, keep_f64=(prec == "f32")))
        v0 = torch.tensor(np.ascontiguousarray(prob.v0).view(np.float64), device="cuda")
        x = torch.randn(ham.dim, dtype=ham.torch_dtype(), device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            tbh.apply_h(ham, x, y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            tbh.apply_h(ham, x, y)
        e1.record()
        torch.cuda.synchronize()
        hx_ms = e0.elapsed_time(e1) / 20
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = tbh.lanczos_eigs(ham, prob.sigma, prob.k, m, v0, reorth=False, n_cand=a.c2_cand)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[prec] = dict(r=r, seconds=dt, hx_ms=hx_ms, hx_GBs=ham.info["hx_bytes"] / hx_ms / 1e6,
                         n_found=r["report"]["n_found"])
        print(f"bench c2: {prec} found {r['report']['n_found']} in {dt:.2f} s", file=sys.stderr, flush=True)
        del ham
    r64, r32 = res["f64"]["r"], res["f32"]["r"]
    errs_raw, errs_ref = [], []
    for e_raw, e_ref in zip(r32["evals"], r32["refined"]):
        if len(r64["refined"]):
            j = int(np.argmin(np.abs(r64["refined"] - e_ref)))
            errs_raw.append(abs(e_raw - r64["refined"][j]))
            errs_ref.append(abs(e_ref - r64["refined"][j]))
    out["value"] = float(max(errs_ref)) if errs_ref else None
    out["extra"] = dict(
        n_found_f32=res["f32"]["n_found"], n_found_f64=res["f64"]["n_found"],
        max_err_raw=float(max(errs_raw)) if errs_raw else None,
        max_err_refined=float(max(errs_ref)) if errs_ref else None,
        max_residual_f32=float(max(r32["res"])) if len(r32["res"]) else None,
        seconds_f32=res["f32"]["seconds"], seconds_f64=res["f64"]["seconds"],
        hx_ms_f32=res["f32"]["hx_ms"], hx_GBs_f32=res["f32"]["hx_GBs"],
        hx_ms_f64=res["f64"]["hx_ms"], hx_GBs_f64=res["f64"]["hx_GBs"],
        evals_f32_refined=[float(v) for v in r32["refined"]],
        evals_f64_refined=[float(v) for v in r64["refined"]])
    print(json.dumps(out), flush=True)


def bench_c4(a):
    """Batched multi-vector H.X: 48 periodic cells (edges 2..12 cells) x 4
    k-points, sp3s* with spin-orbit, 16 complex right-hand vectors, in one
    persistent graph launch (autotuned) against one launch per cell."""
    import torch
    import paper_1003_4570_amd as tbh
    import workloads as W
    print("bench c4: building 192 Hamiltonians", file=sys.stderr, flush=True)
    items = W.c4_batch(0)
    ctx = tbh.Context(0)
    hams, Xs, Ys = [], [], []
    atoms = 0
    for prob, x in items:
        h = tbh.build_hamiltonian(ctx, **tbh.problem_args(prob, multi_vector=True))
        hams.append(h)
        Xs.append(torch.from_numpy(x.astype(np.complex64)).cuda())
        Ys.append(torch.empty_like(Xs[-1]))
        atoms += prob.n_atoms
    b = tbh.Batch(ctx, hams, Xs, Ys)
    if a.c4_grid > 0:
        # a fixed configuration: the trace then holds the batched launches alone
        b.configure(a.c4_grid, a.c4_remap)
        cfg = dict(grid=a.c4_grid, remap=a.c4_remap, ms=None)
    else:
        cfg = b.autotune(None)

    def timeit(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    t_graph = timeit(b.apply)
    t_sep = None if a.c4_batched_only else timeit(b.apply_separate)
    per_atom = 5 * 10 * 10 * 8 + 16 + 2 * 10 * 16 * 8
    byts = per_atom * atoms
    flops = atoms * 2 * (5 * 10 * 10) * 16 * 4     # complex MACs: 4 real multiply-adds
    out = {"metric": "batched multi-vector H.X GB/s", "value": round(byts / t_graph / 1e6, 1), "unit": "GB/s",
           "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "dtype": "f32",
           "config": {"workload": "c4_48cells_x4k_sp3s_so_16rhs", "atom_k_instances": atoms,
                      "bytes_per_apply": byts},
           "extra": dict(ms_graph=t_graph, ms_separate=t_sep,
                         speedup_vs_separate=None if t_sep is None else t_sep / t_graph,
                         autotuned=cfg, tflops=flops / t_graph / 1e9,
                         mfma_fp32_frac=flops / t_graph / 1e9 / 157.3)}
    print(json.dumps(out), flush=True)


def bench_c2sd(a):
    """The 64,000-atom hard-wall SO cube (C2) with spin-diagonal bond storage
    against the stored format: time per fused H.x of 500 Lanczos steps
    (HIP events), the bytes each format reads, and the 16 values nearest
    mid-gap of the full 6000-step solve through each format."""
    import torch
    import paper_1003_4570_amd as tbh
    import workloads as W
    prob = W.c2_hardwall_so(0, m=a.c2_m)
    ctx = tbh.Context(0)
    v0 = torch.tensor(np.ascontiguousarray(prob.v0).view(np.float64), device="cuda")
    res = {}
    for fmt in ("stored", "spin_diagonal"):
        print(f"bench c2sd: build {fmt}", file=sys.stderr, flush=True)
        ham = tbh.build_hamiltonian(ctx, **tbh.problem_args(prob, keep_f64=True,
                                                           spin_diagonal=(fmt == "spin_diagonal")))
        tbh.lanczos_run(ham, ITERS_PER_STEP, v0, reorth=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            a_, b_, _ = tbh.lanczos_run(ham, ITERS_PER_STEP, v0, reorth=False)
        torch.cuda.synchronize()
        step_us = (time.perf_counter() - t0) / (3 * ITERS_PER_STEP) * 1e6
        _, _, rep = tbh.lanczos_run(ham, ITERS_PER_STEP, v0, reorth=False, time_hx=True)
        hx_us = rep["hx_seconds"] / ITERS_PER_STEP * 1e6
        by = ham.info["hx_bytes"] + ham.info["dim"] * 8          # + x_prev (complex FP32)
        print(f"bench c2sd: solve {fmt}", file=sys.stderr, flush=True)
        r = tbh.lanczos_eigs(ham, prob.sigma, 16, a.c2_m, v0, reorth=False, n_cand=a.c2_cand)
        res[fmt] = dict(hx_us=hx_us, step_us=step_us, hx_bytes=by, GBs=by / (hx_us * 1e-6) / 1e9, alpha=a_,
                        refined=np.sort(r["refined"]), n_found=r["report"]["n_found"],
                        solve_s=r["report"]["seconds"])
        del ham
        torch.cuda.empty_cache()
    st, sd = res["stored"], res["spin_diagonal"]
    diff = float(np.abs(st["refined"] - sd["refined"]).max()) if st["n_found"] == sd["n_found"] else None
    out = {"metric": "H.x time per Lanczos step, spin-diagonal bond blocks", "value": round(sd["hx_us"], 2),
           "unit": "us", "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f32",
           "config": {"workload": f"lanczos{a.c2_m}_si20x20x20_hardwall_sp3d5s_so_spin_diagonal",
                      "atoms": prob.n_atoms},
           "extra": {"stored_hx_us": round(st["hx_us"], 2), "hx_speedup": round(st["hx_us"] / sd["hx_us"], 2),
                     "stored_step_us": round(st["step_us"], 2), "spin_diagonal_step_us": round(sd["step_us"], 2),
                     "stored_hx_bytes": st["hx_bytes"], "spin_diagonal_hx_bytes": sd["hx_bytes"],
                     "stored_GBs": round(st["GBs"], 1), "spin_diagonal_GBs": round(sd["GBs"], 1),
                     "spin_diagonal_frac_hbm": round(sd["GBs"] / 8000.0, 4),
                     "stored_solve_s": round(st["solve_s"], 3), "spin_diagonal_solve_s": round(sd["solve_s"], 3),
                     "n_found": [st["n_found"], sd["n_found"]], "max_refined_diff_eV": diff,
                     "max_alpha_diff_vs_stored": float(abs(st["alpha"][:50] - sd["alpha"][:50]).max())}}
    print(json.dumps(out), flush=True)


def bench_c5train(a):
    """Training step of the start-potential surrogate on the 8x8x60-cell
    slab's grid (32 x 32 x 240 nodes, 4 input maps, 6 layers of 32 channels,
    dilations 1,2,4,8,2,1), batch 8 of seeded random maps: time per sample
    and the convolutions' MFMA rate (forward, backward-data and weight
    gradient: 3 x 2 x 27 x C_in x C_out flop per voxel and layer) against
    the FP16 dense peak."""
    import torch
    import paper_1003_4570_amd as tbh
    import workloads as W
    grid = (32, 32, 240)
    nx, ny, nz = grid
    dil = (1, 2, 4, 8, 2, 1)
    ctx = tbh.Context(0)
    net = tbh.Net(ctx, grid, in_channels=4, dilations=dil)
    net.set_params(W.init_surrogate_weights(0, in_channels=4, n_layers=len(dil)))
    g = torch.Generator(device="cpu").manual_seed(0)
    xs = [torch.randn((4, nz, ny, nx), generator=g).float().cuda() for _ in range(8)]
    ts = [torch.randn((nz, ny, nx), generator=g).float().cuda() for _ in range(8)]
    for _ in range(max(1, a.warmup)):
        net.train_step(xs, ts, lr=1e-5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        net.train_step(xs, ts, lr=1e-5)
    torch.cuda.synchronize()
    per_sample = (time.perf_counter() - t0) / (a.steps * len(xs))
    chans = [(4, 32)] + [(32, 32)] * (len(dil) - 2) + [(32, 1)]
    flops = 3 * 2 * 27 * sum(ci * co for ci, co in chans) * nx * ny * nz
    out = {"metric": "surrogate training time per sample", "value": round(per_sample * 1e3, 3), "unit": "ms",
           "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f16 (f32 accumulation)",
           "config": {"workload": "surrogate_train_grid32x32x240_6layers_32ch_batch8"},
           "extra": {"conv_tflops": round(flops / per_sample / 1e12, 2),
                     "mfma_fp16_frac": round(flops / per_sample / 1e12 / 2500.0, 4)}}
    print(json.dumps(out), flush=True)


def bench_c2cgs2(a):
    """Full reorthogonalisation at C2 scale: 500 Lanczos steps with CGS2 on
    the 64,000-atom hard-wall SO cube (FP32 basis of 1.28M complex
    elements).  Step j reads the j basis vectors twice per pass (dots, then
    update) in two passes: 4 j dim 8 bytes, 16 dim m^2 bytes over the run.
    Reports the whole run's rate against those bytes and the H.x share."""
    import torch
    import paper_1003_4570_amd as tbh
    import workloads as W
    m = 500
    prob = W.c2_hardwall_so(0, m=m)
    ctx = tbh.Context(0)
    ham = tbh.build_hamiltonian(ctx, **tbh.problem_args(prob))
    v0 = torch.tensor(np.ascontiguousarray(prob.v0).view(np.float64), device="cuda")
    tbh.lanczos_run(ham, 50, v0, reorth=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, rep = tbh.lanczos_run(ham, m, v0, reorth=True, time_hx=True)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    dim = ham.info["dim"]
    reorth_bytes = sum(4 * j * dim * 8 for j in range(1, m + 1))
    reorth_s = sec - rep["hx_seconds"]
    out = {"metric": "CGS2 reorthogonalisation GB/s (algorithmic)", "value": round(reorth_bytes / reorth_s / 1e9, 1),
           "unit": "GB/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "dtype": "f32 basis, f64 sums",
           "config": {"workload": "lanczos500_cgs2_si20x20x20_hardwall_sp3d5s_so", "dim": dim, "steps": m},
           "extra": {"seconds": round(sec, 3), "hx_seconds": round(rep["hx_seconds"], 4),
                     "reorth_bytes": reorth_bytes, "frac_hbm": round(reorth_bytes / reorth_s / 8e12, 4)}}
    print(json.dumps(out), flush=True)


def bench_c3t(a):
    """The million-atom alloy with tabulated bond blocks (an unstrained real
    H at Gamma has one block per sublattice, species pair and slot): time per
    H.x and per Lanczos step against the stored-block format, 500 steps."""
    import torch
    import paper_1003_4570_amd as tbh
    import workloads as W
    prob = W.c3_alloy(0)
    ctx = tbh.Context(0)
    v0 = torch.tensor(prob.v0, dtype=torch.float64, device="cuda")
    res = {}
    for fmt in ("stored", "tabulated"):
        print(f"bench c3t: build {fmt}", file=sys.stderr, flush=True)
        ham = tbh.build_hamiltonian(ctx, **tbh.problem_args(prob, tabulated=(fmt == "tabulated")))
        tbh.lanczos_run(ham, ITERS_PER_STEP, v0, reorth=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            a_, b_, _ = tbh.lanczos_run(ham, ITERS_PER_STEP, v0, reorth=False)
        torch.cuda.synchronize()
        step_us = (time.perf_counter() - t0) / (3 * ITERS_PER_STEP) * 1e6
        _, _, rep = tbh.lanczos_run(ham, ITERS_PER_STEP, v0, reorth=False, time_hx=True)
        hx_us = rep["hx_seconds"] / ITERS_PER_STEP * 1e6
        # fused step bytes: the format's H.x bytes plus x_prev
        by = ham.info["hx_bytes"] + ham.info["dim"] * 4
        res[fmt] = dict(hx_us=hx_us, step_us=step_us, hx_bytes=by, GBs=by / (hx_us * 1e-6) / 1e9,
                        alpha=a_, beta=b_)
        del ham
    st, tb = res["stored"], res["tabulated"]
    out = {"metric": "H.x time per Lanczos step, tabulated bond blocks", "value": round(tb["hx_us"], 2),
           "unit": "us", "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f32",
           "config": {"workload": "lanczos500_si0.7ge0.3_51x51x51_sp3d5s_fp32_tabulated", "atoms": prob.n_atoms},
           "extra": {"stored_hx_us": round(st["hx_us"], 2), "hx_speedup": round(st["hx_us"] / tb["hx_us"], 2),
                     "stored_step_us": round(st["step_us"], 2), "tabulated_step_us": round(tb["step_us"], 2),
                     "step_speedup": round(st["step_us"] / tb["step_us"], 2),
                     "tabulated_hx_bytes": tb["hx_bytes"], "tabulated_GBs": round(tb["GBs"], 1),
                     "tabulated_frac_hbm": round(tb["GBs"] / 8000.0, 4),
                     "max_alpha_diff_vs_stored": float(abs(st["alpha"][:50] - tb["alpha"][:50]).max())}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--workload", default="c3", choices=["c3", "c2", "c4", "c3t", "c2sd", "c5train", "c2cgs2"],
                    help="c3: H.x GB/s in Lanczos (default); c2: FP32 vs FP64 eigenvalues; "
                         "c4: batched multi-vector H.X; c3t: the c3 alloy with tabulated bond blocks; "
                         "c2sd: c2 with spin-diagonal bond blocks; c5train: surrogate training step; "
                         "c2cgs2: full reorthogonalisation at c2 scale")
    ap.add_argument("--no-scf", action="store_true", help="skip the SCF learned-vs-zero-start leg")
    ap.add_argument("--scf-layouts", type=int, default=2, help="held-out donor layouts of the SCF leg")
    ap.add_argument("--c4-grid", type=int, default=0, help="c4: fixed persistent grid (0 = autotune)")
    ap.add_argument("--c4-remap", type=int, default=2, help="c4: atom walk with --c4-grid (0, 1 or 2)")
    ap.add_argument("--c4-batched-only", action="store_true", help="c4: skip the one-launch-per-cell timing")
    ap.add_argument("--c2-m", type=int, default=6000)
    ap.add_argument("--c2-cand", type=int, default=256)
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported (single-GPU build)",
              file=sys.stderr)
        sys.exit(2)
    if a.calibrate_copy:
        calibrate_copy()
        return
    if a.workload == "c2":
        bench_c2(a)
        return
    if a.workload == "c4":
        bench_c4(a)
        return
    if a.workload == "c2cgs2":
        bench_c2cgs2(a)
        return
    if a.workload == "c5train":
        bench_c5train(a)
        return
    if a.workload == "c2sd":
        bench_c2sd(a)
        return
    if a.workload == "c3t":
        bench_c3t(a)
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
    hx_bytes_layout = ham.info["hx_bytes"] + ham.info["dim"] * 4
    # method bytes (no layout padding): bonds, diagonal on-site, neighbours, x, y, x_prev per atom
    hx_bytes = C3_METHOD_BYTES_PER_ATOM * ham.info["n_atoms"]
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
                   "hx_bytes_per_launch": hx_bytes, "hx_bytes_per_launch_with_layout_padding": hx_bytes_layout},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "hx_kernel<float,real,10,10,diag,lanczos>",
                     "avg_launch_ms": round(hx_avg * 1e3, 4)},
    }
    out["roofline"]["frac_with_layout_padding"] = round(hx_bytes_layout / hx_avg / 1e9 / HBM_PEAK_GBS, 4)
    if not a.no_scf:
        # the second half of the metric: SCF time-to-converge, learned vs zero start
        out["scf_learned_vs_plain"] = scf_leg(tuple(range(1000, 1000 + a.scf_layouts)))
    if not a.no_cpu_baseline:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
