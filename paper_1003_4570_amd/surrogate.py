"""Learned start potential for the self-consistent loop.

    python -m paper_1003_4570_amd.surrogate --geometry c5 gen   --out DIR --seeds 0:100
    python -m paper_1003_4570_amd.surrogate --geometry c5 pack  --out DATA.npz DIR [DIR ...]
    python -m paper_1003_4570_amd.surrogate --geometry c5 train --data DATA.npz --out W.npz
    python -m paper_1003_4570_amd.surrogate --geometry c5 eval  --weights W.npz --seeds 1000:1016

The self-consistent Schrodinger-Poisson loop (Sec. III-A) is run by the
library (tbh_scf_*), and so is every step of the learned start: building the
network's input maps, the forward passes, the average over the slab's point
operations, forming U0 and the fallback to the zero start
(tbh_scf_set_start).  This module orchestrates: it generates converged
solutions with the plain method (zero start, linear mixing), trains the
convolutional surrogate on them with the library's device kernels
(tbh_net_*), and compares SCF time-to-converge from the zero start, the
training-mean start and the learned start on held-out donor layouts.

The network (by default four layers; deeper dilation lists are supported)
sees four maps on the a/4 grid: the donor count, the two sublattice
occupation masks (a diamond lattice fills only one node in eight, and which
nodes it fills is not invariant under a one-node shift, so without them a
convolution cannot tell an atom site from an empty node) and the electron
potential energy of the bare donor charge (the Poisson solution of the donors
alone in the dielectric, divided by a fixed scale), which carries the
long-range part the network's finite receptive field cannot reach.  Its
target is the electron part E = U* - U_bare of the converged potential.  The
zero start stays the fallback: a start is abandoned (and the loop restarted
from zero) when the residual turns non-finite, grows three steps in a row,
or the first residual exceeds ten times the zero start's.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

import paper_1003_4570_amd as tbh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

N_IN = 4   # input maps: donor count, A and B sublattice masks, bare-donor potential

# The loop's settings per geometry.  The study slab (3x3x8 cells, 576 atoms)
# keeps the Lanczos eigen-solve (64 candidates of 800 CGS2 steps); the
# 8x8x60-cell delta-doped slab (30,720 atoms) uses the filtered block solver
# (a block of 64 states, folded Chebyshev filters, warm-started every step).
# The first eigen-solve, from a random block, does not reach 0.01 eV in 60
# filter passes on this slab.  From the zero start with linear mixing it
# stops after 30 (the library applies filter_max_iter_cold to that case
# only): measured on 8 held-out layouts, 60 -> 30 passes for every start
# took the zero start from 1.92 to 1.70 s but the learned start from 101.5
# to 107 steps, and the Newton-Raphson runs from 2.22 / 1.27 s to
# 2.64 / 1.34 s (zero / learned).
GEOMETRIES = {
    "study": dict(problem=W.study_slab,
                  scf=dict(mix_alpha=0.05, tol_eV=1e-4, n_cand=64, lanczos_iter=800, res_tol=1e-4, T_K=4.0,
                           eps_r=11.7)),
    "c5": dict(problem=W.c5_slab,
               scf=dict(mix_alpha=0.05, tol_eV=1e-4, res_tol=1e-4, T_K=4.0, eps_r=11.7, eig_mode=1, block=64,
                        filter_degree=20, filter_degree_cold=80, filter_max_iter=60, filter_max_iter_cold=30,
                        k_states=40)),
}
SCF_DEFAULTS = GEOMETRIES["study"]["scf"]


def _seeds(spec):
    a, b = spec.split(":")
    return list(range(int(a), int(b)))


class Start:
    """A trained start: the network (library handle), the training mean of
    the target on the device, its scale, the input scale and the target kind
    ("E": U* minus the bare-donor potential; "U": U* itself)."""

    def __init__(self, study, weights):
        import torch
        wz = np.load(weights)
        nz, ny, nx = wz["Tbar"].shape
        dil = tuple(int(d) for d in wz["dilations"]) if "dilations" in wz.files else (1, 2, 4, 1)
        self.net = tbh.Net(study.ctx, (nx, ny, nz), in_channels=N_IN, dilations=dil)
        self.net.set_params(wz["params"])
        self.Tbar = torch.from_numpy(np.asarray(wz["Tbar"], dtype=np.float32)).cuda()
        self.scale = float(wz["scale"])
        self.feat_scale = float(wz["feat_scale"])
        self.target = str(wz["target"])
        self.train_seeds = set(int(v) for v in wz["train_seeds"])
        if self.target != "E":
            raise ValueError("the device start builds U_bare + mean + scale * net: weights with target E")


class Study:
    """One Hamiltonian shared by every donor layout of a slab geometry (the
    layouts differ in their donor sites and Lanczos start vector only)."""

    def __init__(self, ctx=None, geometry="study", **scf_kw):
        import torch
        self.ctx = ctx or tbh.Context(0)
        self.geometry = geometry
        G = GEOMETRIES[geometry]
        self.problem = G["problem"]
        p0 = self.problem(0)
        self.grid = p0.extra["grid"]
        self.gap = p0.extra["gap"]
        self.pos_q = p0.pos_q
        self.kw = dict(G["scf"])
        if self.kw.get("eig_mode", 0) == 1:
            self.kw["e_vbm"] = self.gap["vbm"]
        self.kw.update(scf_kw)
        multi = self.kw.get("eig_mode", 0) == 1
        self.ham = tbh.build_hamiltonian(self.ctx, **tbh.problem_args(p0, prec="f32", keep_f64=True,
                                                                      multi_vector=multi))
        self.torch = torch

    def scf(self, seed, **over):
        p = self.problem(seed)
        s = tbh.SCF(self.ham, self.grid, p.extra["donor_atoms"], p.v0, self.gap["mid"], self.gap["cbm"],
                    W.H_GRID_NM, **{**self.kw, **over})
        return s, p

    def donor_map(self, p):
        return W.donor_map(p.pos_q, p.extra["donor_atoms"], self.grid)

    def bare_potential(self, dmap):
        """Electron potential energy (eV, device FP64 [nz, ny, nx]) of the
        donor charge alone: -phi with -eps0 eps_r Lap_h phi = donors / h^3."""
        torch = self.torch
        rho = torch.from_numpy(np.asarray(dmap, dtype=np.float64) / W.H_GRID_NM ** 3).cuda()
        phi, _, rel = tbh.poisson_solve(self.ctx, self.grid, W.H_GRID_NM, self.kw["eps_r"], rho, rel_tol=1e-12)
        if not rel <= 1e-10:
            raise RuntimeError(f"bare-donor Poisson solve did not converge (relative residual {rel})")
        return -phi

    def electron_potential(self, n_atoms):
        """Potential energy of the electrons (eV, device FP64 map) for the
        electrons per atom n (device FP64, caller order): with rho = -e n / h^3
        on the atom nodes, U_e = -phi(rho); U* = U_bare + U_e at the fixed point."""
        torch = self.torch
        nx, ny, nz = self.grid
        q = torch.from_numpy(self.pos_q.astype(np.int64)).cuda()
        nmap = torch.zeros((nz, ny, nx), dtype=torch.float64, device="cuda")
        nmap.index_put_((q[:, 2], q[:, 1], q[:, 0]), n_atoms.double(), accumulate=True)
        phi, _, rel = tbh.poisson_solve(self.ctx, self.grid, W.H_GRID_NM, self.kw["eps_r"],
                                        (nmap / W.H_GRID_NM ** 3).contiguous(), rel_tol=1e-12)
        if not rel <= 1e-10:
            raise RuntimeError(f"electron Poisson solve did not converge (relative residual {rel})")
        return phi

    def inputs(self, dmap, feat_scale):
        """The network's input maps, float32 [4, nz, ny, nx] on the device
        (training; at inference the library builds the same maps itself)."""
        torch = self.torch
        if not hasattr(self, "_masks"):
            self._masks = torch.from_numpy(W.sublattice_masks(self.pos_q, self.grid)).cuda()
        d = torch.from_numpy(np.asarray(dmap, dtype=np.float32)).cuda()
        ub = (self.bare_potential(dmap) / feat_scale).float()
        return torch.stack([d, self._masks[0], self._masks[1], ub]).contiguous()

    def surrogate(self, weights):
        return Start(self, weights)

    def run(self, seed, start=None, max_iter=400, first_res_limit=0.0, mean_only=False, fixed_start=None, **over):
        """SCF of one layout from the zero start (start None), the mean start
        (start and mean_only) or the learned start (start), the start built
        by the library (tbh_scf_set_start, its time included), or from an
        explicit FP32 device map added to U_bare as the mean start
        (fixed_start: a test of the fallback); over: loop options that
        replace the geometry's (e.g. update_mode=1).  Returns the record
        (iterations, seconds, residuals, converged, fell_back, U, U0)."""
        torch = self.torch
        s, p = self.scf(seed, **over)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if fixed_start is not None:
            s.set_start("mean", mean=fixed_start, first_res_limit=first_res_limit)
        elif start is None:
            s.set_start("zero")
        elif mean_only:
            s.set_start("mean", mean=start.Tbar, first_res_limit=first_res_limit)
        else:
            s.set_start("learned", net=start.net, mean=start.Tbar, scale=start.scale,
                        feat_scale=start.feat_scale, symmetrize=True, first_res_limit=first_res_limit)
        torch.cuda.synchronize()
        t_start = time.perf_counter() - t0
        U0 = s.potential()
        t1 = time.perf_counter()
        res, fell = [], False
        it = 0
        r = None
        while it < max_iter:
            r = s.step()
            it += 1
            res.append(r["residual"])
            fell = fell or bool(r["fell_back"])
            if r["converged"]:
                break
        torch.cuda.synchronize()
        dt = t_start + (time.perf_counter() - t1)
        U = s.potential()
        n = s.density() if it else None
        s.close()
        return dict(seed=seed, iterations=it, seconds=dt, start_seconds=t_start, residuals=res,
                    converged=bool(r is not None and r["converged"]), fell_back=fell, U=U, U0=U0, n=n)


def generate(out_dir, seeds, max_iter=400, budget_s=None, geometry="study"):
    """Plain-method (zero start) SCF runs; per converged layout the electrons
    per atom (float32, caller order; the converged potential is U_bare plus
    their Poisson potential), iterations and seconds."""
    os.makedirs(out_dir, exist_ok=True)
    st = Study(geometry=geometry)
    t0 = time.perf_counter()
    for sd in seeds:
        if budget_s is not None and time.perf_counter() - t0 > budget_s:
            print(json.dumps(dict(stopped_at_seed=sd, reason="time budget")), flush=True)
            break
        if os.path.exists(os.path.join(out_dir, f"layout_{sd:05d}.npz")):
            continue
        rec = st.run(sd, None, max_iter)
        np.savez(os.path.join(out_dir, f"layout_{sd:05d}.npz"), n=rec["n"].float().cpu().numpy(),
                 iterations=rec["iterations"], seconds=rec["seconds"], converged=rec["converged"])
        print(json.dumps(dict(seed=sd, iterations=rec["iterations"], seconds=round(rec["seconds"], 3),
                              converged=rec["converged"])), flush=True)


def pack(out_path, sources):
    """Merge converged layouts (per-layout files written by generate() or
    packed files) into one compressed .npz: seeds, n (electrons per atom,
    float32 [layouts, atoms]), iterations, seconds.  A seed seen twice keeps
    its last copy."""
    acc = {}
    for src in sources:
        if os.path.isdir(src):
            for fn in sorted(os.listdir(src)):
                if not (fn.startswith("layout_") and fn.endswith(".npz")):
                    continue
                d = np.load(os.path.join(src, fn))
                if bool(d["converged"]):
                    acc[int(fn[7:12])] = (d["n"].astype(np.float32), int(d["iterations"]), float(d["seconds"]))
        else:
            d = np.load(src)
            for i, sd in enumerate(d["seeds"]):
                acc[int(sd)] = (d["n"][i], int(d["iterations"][i]), float(d["seconds"][i]))
    keys = sorted(acc)
    np.savez_compressed(out_path, seeds=np.array(keys), n=np.stack([acc[k][0] for k in keys]),
                        iterations=np.array([acc[k][1] for k in keys]),
                        seconds=np.array([acc[k][2] for k in keys]))
    return len(keys)


def load_dataset(path, study):
    """Donor maps, bare-donor potentials and electron potentials (targets) of
    the packed layouts: float32 donor maps [n, nz, ny, nx], device FP64 maps,
    seeds."""
    torch = study.torch
    d = np.load(path)
    seeds = [int(v) for v in d["seeds"]]
    X = np.stack([study.donor_map(study.problem(sd)) for sd in seeds])
    Ub = torch.stack([study.bare_potential(x) for x in X])
    E = torch.stack([study.electron_potential(torch.from_numpy(n).cuda()) for n in d["n"]])
    return X, Ub, E, seeds


def lattice_shifts(grid):
    """In-plane translations of the diamond lattice that map the periodic
    cell onto itself, as (sx, sy) on the a/4 grid: both even, sum divisible
    by 4 (generated by the fcc vectors (2, 2, 0) and (4, 0, 0))."""
    nx, ny, _ = grid
    return [(sx, sy) for sy in range(0, ny, 2) for sx in range(0, nx, 2) if (sx + sy) % 4 == 0]


def point_ops():
    """The in-plane point operations that map the diamond slab onto itself
    (its two sublattices each onto itself): identity, the (110) mirror
    (x, y) -> (y, x), the (1-10) mirror (x, y) -> (-y, -x) and their product,
    the two-fold rotation (x, y) -> (-x, -y), all about the atom at the
    origin, on maps whose last two axes are (y, x).  Pairs (op, inverse);
    each is its own inverse."""
    import torch

    def ident(a):
        return a

    def mirror(a):
        return a.transpose(-1, -2)

    def rot2(a):
        return torch.roll(torch.flip(a, dims=(-1, -2)), shifts=(1, 1), dims=(-2, -1))

    def antimirror(a):
        return rot2(a).transpose(-1, -2)

    return [(ident, ident), (mirror, mirror), (antimirror, antimirror), (rot2, rot2)]


def symmetrize(a, grid):
    """Average of the [.., nz, ny, nx] map over the lattice translations."""
    return np.mean([np.roll(a, (sy, sx), axis=(-2, -1)) for sx, sy in lattice_shifts(grid)], axis=0)


def near_plane_weights(study, donor_z, near_weight, half_width=3):
    """Loss weights 1 + near_weight on atom nodes within half_width grid
    planes of the donor plane (where the start error is largest), 1
    elsewhere; float32 [nz, ny, nx]."""
    nx, ny, nz = study.grid
    m = W.sublattice_masks(study.pos_q, study.grid).sum(axis=0) > 0
    z = np.arange(nz)[:, None, None]
    return (1.0 + near_weight * (m & (np.abs(z - donor_z) <= half_width))).astype(np.float32)


def train(data, out_path, epochs=300, lr=1e-3, batch=8, seed=0, n_val=0, ctx=None, dilations=(1, 2, 4, 1),
          near_weight=0.0, geometry="study", time_budget=None, warmup=0, init=None):
    """Fit the network to the electron part E = U* - U_bare of converged
    potentials (added back to the exact U_bare at inference).  The targets
    are taken relative to their training mean averaged over the lattice
    translations (an exact symmetry of the donor ensemble) and divided by
    their RMS over the nodes where they vary between layouts, and every epoch
    shows each layout under a random lattice translation.  near_weight > 0
    weights the loss on the atoms next to the donor plane.  The last n_val
    layouts are held out, their max-norm start error reported every 25
    epochs, and the parameters with the lowest median of it are the ones
    saved.  The learning rate rises linearly over the first warmup epochs and
    follows a cosine decay from lr to zero (over epochs, or over time_budget
    seconds when given).  init: a saved network whose parameters, mean and
    scales the training continues from (same geometry and layers)."""
    import torch
    st = Study(ctx, geometry=geometry)
    X, Ub, E, seeds = load_dataset(data, st)
    grid = st.grid
    feat_scale = float(Ub.std())
    ntr = len(X) - n_val
    Tbar = symmetrize(E[:ntr].mean(dim=0).cpu().numpy(), grid)
    if init is not None:
        w0 = np.load(init)
        feat_scale = float(w0["feat_scale"])
        Tbar = w0["Tbar"].astype(np.float64)
    Tbar_d = torch.from_numpy(Tbar).cuda()
    # target scale: the spread of the electron part where it varies between
    # layouts (near the donor plane; far from it every layout has the same
    # potential and the map is zero), so that the targets are O(1) there
    dev = E[:ntr] - Tbar_d
    vox_sd = dev.std(dim=0)
    live = vox_sd > 1e-2 * vox_sd.max()
    scale = float(dev[:, live].pow(2).mean().sqrt()) if init is None else float(np.load(init)["scale"])
    T = ((E - Tbar_d) / scale).float()
    nz, ny, nx = X.shape[1:]
    net = tbh.Net(st.ctx, (nx, ny, nz), in_channels=N_IN, dilations=dilations)
    net.set_params(W.init_surrogate_weights(seed, in_channels=N_IN, n_layers=len(dilations)) if init is None
                   else np.load(init)["params"])
    if near_weight > 0:
        donor_z = int(np.flatnonzero(X.sum(axis=(0, 2, 3)))[0])
        net.set_loss_weights(torch.from_numpy(near_plane_weights(st, donor_z, near_weight)).cuda())
    Xd = [st.inputs(x, feat_scale) for x in X]
    Td = [t.contiguous() for t in T]
    shifts = lattice_shifts(grid)
    rng = np.random.default_rng(seed)

    def val_errors():
        e = []
        for i in range(ntr, len(X)):
            u = Tbar_d + scale * net.forward(Xd[i]).double()
            e.append(float((u - E[i]).abs().max()))
        return e

    hist = []
    skipped = 0
    best = (np.inf, None, -1)    # validation median, parameters, epoch
    t0 = time.perf_counter()
    for ep in range(epochs):
        frac = ep / epochs if time_budget is None else min(1.0, (time.perf_counter() - t0) / time_budget)
        # linear warm-up over the first warmup epochs, then cosine decay
        lr_ep = 0.5 * lr * (1.0 + np.cos(np.pi * frac)) * min(1.0, (ep + 1) / max(1, warmup))
        order = rng.permutation(ntr)
        tot = 0.0
        for b0 in range(0, len(order), batch):
            idx = order[b0:b0 + batch]
            xs, ts = [], []
            for i in idx:
                sx, sy = shifts[rng.integers(len(shifts))]
                xs.append(torch.roll(Xd[i], (sy, sx), dims=(2, 3)).contiguous())
                ts.append(torch.roll(Td[i], (sy, sx), dims=(1, 2)).contiguous())
            loss = net.train_step(xs, ts, lr=lr_ep)
            if np.isfinite(loss):
                tot += loss * len(idx)
            else:
                skipped += 1           # the library skipped the update
        hist.append(tot / len(order))
        done = time_budget is not None and time.perf_counter() - t0 > time_budget
        if ep % 25 == 0 or ep == epochs - 1 or done:
            rec = dict(epoch=ep, loss=hist[-1], lr=lr_ep, seconds=round(time.perf_counter() - t0, 1),
                       skipped_steps=skipped)
            if n_val:
                ve = val_errors()
                rec.update(val_err_median=float(np.median(ve)), val_err_max=float(np.max(ve)))
                if np.median(ve) < best[0]:
                    best = (float(np.median(ve)), net.get_params(), ep)
            print(json.dumps(rec), flush=True)
        if done:
            break
    torch.cuda.synchronize()
    params = net.get_params()
    if best[1] is not None:
        # the checkpoint with the lowest validation error
        params = best[1]
        print(json.dumps(dict(kept_epoch=best[2], val_err_median=best[0])), flush=True)
    prior_s, prior_ep = 0.0, 0
    if init is not None:
        w0 = np.load(init)
        prior_s, prior_ep = float(w0["train_seconds"]), int(w0["epochs"])
    np.savez(out_path, params=params, Tbar=Tbar.astype(np.float32), scale=scale, feat_scale=feat_scale,
             target="E", dilations=np.array(dilations), near_weight=near_weight, loss=np.array(hist),
             train_seeds=np.array(seeds[:ntr]), train_seconds=prior_s + time.perf_counter() - t0, geometry=geometry,
             epochs=prior_ep + len(hist))
    return hist


def evaluate(weights, seeds, max_iter=400, ctx=None, with_mean=True, geometry="study", newton=False):
    """Per held-out layout: SCF from the zero start, from the mean start (the
    network's output replaced by zero: the symmetrized training mean plus
    the bare-donor potential) and from the learned start, each start built
    by the library with its time included; the fallback limit is ten times
    the zero start's first residual.  newton: also the zero and learned
    starts with the Newton-Raphson update in place of linear mixing."""
    st = Study(ctx, geometry=geometry)
    start = st.surrogate(weights)
    out = []
    for sd in seeds:
        zero = st.run(sd, None, max_iter)
        Ustar = zero["U"]
        lim = 10.0 * zero["residuals"][0]
        rec = dict(seed=sd, zero=dict(iterations=zero["iterations"], seconds=zero["seconds"],
                                      converged=zero["converged"]),
                   zero_err0=float(Ustar.abs().max()))
        if with_mean:
            mean = st.run(sd, start, max_iter, lim, mean_only=True)
            rec["mean"] = dict(iterations=mean["iterations"], seconds=mean["seconds"], converged=mean["converged"],
                               fell_back=mean["fell_back"], err0=float((mean["U0"] - Ustar).abs().max()))
        learned = st.run(sd, start, max_iter, lim)
        rec["learned"] = dict(iterations=learned["iterations"], seconds=learned["seconds"],
                              start_seconds=learned["start_seconds"], converged=learned["converged"],
                              fell_back=learned["fell_back"], err0=float((learned["U0"] - Ustar).abs().max()),
                              fixed_point_diff=float((learned["U"] - Ustar).abs().max()))
        if newton:
            for kind, sta in (("zero_newton", None), ("learned_newton", start)):
                r = st.run(sd, sta, max_iter, lim if sta is not None else 0.0, update_mode=1)
                rec[kind] = dict(iterations=r["iterations"], seconds=r["seconds"], converged=r["converged"],
                                 fell_back=r["fell_back"], fixed_point_diff=float((r["U"] - Ustar).abs().max()))
        out.append(rec)
        print(json.dumps(rec), flush=True)
    return out


def summarize(records):
    def med(key, sub):
        return float(np.median([r[key][sub] for r in records]))
    s = dict(n=len(records), zero_iters=med("zero", "iterations"), learned_iters=med("learned", "iterations"),
             zero_s=med("zero", "seconds"), learned_s=med("learned", "seconds"),
             speedup_time=med("zero", "seconds") / med("learned", "seconds"),
             speedup_iters=med("zero", "iterations") / med("learned", "iterations"),
             learned_err0=med("learned", "err0"),
             zero_err0=float(np.median([r["zero_err0"] for r in records])),
             fallbacks=int(sum(r["learned"]["fell_back"] for r in records)))
    for kind in ("zero_newton", "learned_newton"):
        if all(kind in r for r in records):
            s[kind + "_iters"] = med(kind, "iterations")
            s[kind + "_s"] = med(kind, "seconds")
    if all("mean" in r for r in records):
        s.update(mean_iters=med("mean", "iterations"), mean_s=med("mean", "seconds"),
                 mean_err0=med("mean", "err0"))
    return s


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--geometry", choices=sorted(GEOMETRIES), default="study")
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("gen")
    g.add_argument("--out", required=True)
    g.add_argument("--seeds", default="0:96")
    g.add_argument("--max-iter", type=int, default=400)
    g.add_argument("--budget", type=float, default=None, help="stop starting layouts after this many seconds")
    k = sub.add_parser("pack")
    k.add_argument("--out", required=True)
    k.add_argument("sources", nargs="+", help="layout directories or packed files")
    t = sub.add_parser("train")
    t.add_argument("--data", required=True, help="packed layouts (pack)")
    t.add_argument("--out", required=True)
    t.add_argument("--epochs", type=int, default=300)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--batch", type=int, default=8)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--val", type=int, default=0, help="hold out this many layouts and report their start error")
    t.add_argument("--dilations", default="1,2,4,1", help="one dilation per layer")
    t.add_argument("--near-weight", type=float, default=0.0,
                   help="extra loss weight on the atoms next to the donor plane")
    t.add_argument("--budget", type=float, default=None, help="stop training after this many seconds")
    t.add_argument("--warmup", type=int, default=0, help="epochs of linear learning-rate warm-up")
    t.add_argument("--init", default=None, help="continue from these saved weights")
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--seeds", default="1000:1016")
    e.add_argument("--no-mean", action="store_true", help="skip the mean-start runs")
    e.add_argument("--newton", action="store_true", help="also run both starts with the Newton-Raphson update")
    e.add_argument("--out", default=None)
    a = ap.parse_args()
    if a.cmd == "gen":
        generate(a.out, _seeds(a.seeds), a.max_iter, a.budget, geometry=a.geometry)
    elif a.cmd == "pack":
        print(json.dumps(dict(layouts=pack(a.out, a.sources))), flush=True)
    elif a.cmd == "train":
        train(a.data, a.out, a.epochs, a.lr, a.batch, a.seed, a.val,
              dilations=tuple(int(v) for v in a.dilations.split(",")), near_weight=a.near_weight,
              geometry=a.geometry, time_budget=a.budget, warmup=a.warmup, init=a.init)
    else:
        recs = evaluate(a.weights, _seeds(a.seeds), with_mean=not a.no_mean, geometry=a.geometry, newton=a.newton)
        s = summarize(recs)
        print(json.dumps(dict(summary=s)), flush=True)
        if a.out:
            with open(a.out, "w") as f:
                json.dump(dict(records=recs, summary=s), f, indent=1)


if __name__ == "__main__":
    main()
