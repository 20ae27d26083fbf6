"""Learned start potential for the self-consistent loop.

    python -m paper_1003_4570_amd.surrogate gen   --out DIR --seeds 0:96
    python -m paper_1003_4570_amd.surrogate pack  --out DATA.npz DIR [DIR ...]
    python -m paper_1003_4570_amd.surrogate train --data DIR --out W.npz [--target U|E]
    python -m paper_1003_4570_amd.surrogate eval  --weights W.npz --seeds 1000:1016

The self-consistent Schrodinger-Poisson loop (Sec. III-A) is run by the
library (tbh_scf_*); this module drives it: it generates converged
potentials with the plain method (zero start, linear mixing), trains the
convolutional surrogate on them with the library's device kernels
(tbh_net_*), and compares SCF time-to-converge from the zero start, the
training-mean start and the learned start on held-out donor layouts.

The network (by default four layers; deeper dilation lists are supported)
sees four maps on the a/4 grid: the donor count, the two
sublattice occupation masks (a diamond lattice fills only one node in eight,
and which nodes it fills is not invariant under a one-node shift, so without
them a convolution cannot tell an atom site from an empty node) and the
electron potential energy of the bare donor charge (the Poisson solution of
the donors alone in the dielectric, divided by a fixed scale), which carries
the long-range part the network's finite receptive field cannot reach.  The
zero start stays the fallback: a learned start is abandoned (and the loop
restarted from zero) when the potential turns non-finite, the residual grows
three steps in a row, or the first residual exceeds ten times the zero
start's.
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

SCF_DEFAULTS = dict(mix_alpha=0.05, tol_eV=1e-4, n_cand=64, lanczos_iter=800, res_tol=1e-4, T_K=4.0,
                    eps_r=11.7)


def _seeds(spec):
    a, b = spec.split(":")
    return list(range(int(a), int(b)))


class Study:
    """One Hamiltonian shared by every donor layout of the study slab."""

    def __init__(self, ctx=None, **scf_kw):
        import torch
        self.ctx = ctx or tbh.Context(0)
        p0 = W.study_slab(0)
        self.grid = p0.extra["grid"]
        self.gap = p0.extra["gap"]
        self.ham = tbh.build_hamiltonian(self.ctx, **tbh.problem_args(p0, prec="f32", keep_f64=True))
        self.kw = dict(SCF_DEFAULTS)
        self.kw.update(scf_kw)
        self.torch = torch

    def scf(self, seed):
        p = W.study_slab(seed)
        s = tbh.SCF(self.ham, self.grid, p.extra["donor_atoms"], p.v0, self.gap["mid"], self.gap["cbm"],
                    W.H_GRID_NM, **self.kw)
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

    def inputs(self, dmap, feat_scale):
        """The network's input maps, float32 [4, nz, ny, nx] on the device."""
        torch = self.torch
        if not hasattr(self, "_masks"):
            self._masks = torch.from_numpy(W.sublattice_masks(W.study_slab(0).pos_q, self.grid)).cuda()
        d = torch.from_numpy(np.asarray(dmap, dtype=np.float32)).cuda()
        ub = (self.bare_potential(dmap) / feat_scale).float()
        return torch.stack([d, self._masks[0], self._masks[1], ub]).contiguous()

    def surrogate(self, weights, symmetrize_output=True):
        """Load trained weights; returns start(dmap) -> device FP64 [nz, ny, nx].
        With symmetrize_output the network's output is averaged over the
        in-plane point operations of the slab (point_ops): each is applied
        to the input maps, the output mapped back, and the four averaged."""
        wz = np.load(weights)
        nz, ny, nx = wz["Tbar"].shape
        dil = tuple(int(d) for d in wz["dilations"]) if "dilations" in wz.files else (1, 2, 4, 1)
        net = tbh.Net(self.ctx, (nx, ny, nz), in_channels=N_IN, dilations=dil)
        net.set_params(wz["params"])
        Tbar = self.torch.from_numpy(wz["Tbar"]).cuda()
        scale, fs, target = float(wz["scale"]), float(wz["feat_scale"]), str(wz["target"])

        def start(dmap):
            x = self.inputs(dmap, fs)
            if symmetrize_output:
                y = sum(inv(net.forward(op(x).contiguous())) for op, inv in point_ops()) / 4.0
            else:
                y = net.forward(x)
            u = Tbar + scale * y.double()
            return u + self.bare_potential(dmap) if target == "E" else u
        start.Tbar = Tbar
        start.target = target
        start.train_seeds = set(int(v) for v in wz["train_seeds"])
        return start

    def run(self, seed, U0=None, max_iter=400, first_res_ref=None, fallback=False):
        """SCF from U0 (device [nz,ny,nx] FP64 or None = zero).  Returns the
        record (iterations, seconds, residuals, converged, fell_back, U)."""
        torch = self.torch
        s, p = self.scf(seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.set_potential(U0)
        res, fell, grow = [], False, 0
        it = 0
        while it < max_iter:
            r = s.step()
            it += 1
            res.append(r["residual"])
            if r["converged"]:
                break
            if fallback and not fell:
                bad = not np.isfinite(r["residual"])
                if len(res) >= 2 and res[-1] > res[-2]:
                    grow += 1
                else:
                    grow = 0
                if len(res) == 1 and first_res_ref is not None and res[0] > 10 * first_res_ref:
                    bad = True
                if bad or grow >= 3:
                    fell = True
                    s.set_potential(None)
                    res.append(float("nan"))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        U = s.potential()
        s.close()
        return dict(seed=seed, iterations=it, seconds=dt, residuals=res, converged=bool(res and res[-1] < self.kw["tol_eV"]),
                    fell_back=fell, U=U)


def generate(out_dir, seeds, max_iter=400, budget_s=None):
    os.makedirs(out_dir, exist_ok=True)
    st = Study()
    t0 = time.perf_counter()
    for sd in seeds:
        if budget_s is not None and time.perf_counter() - t0 > budget_s:
            print(json.dumps(dict(stopped_at_seed=sd, reason="time budget")), flush=True)
            break
        if os.path.exists(os.path.join(out_dir, f"layout_{sd:05d}.npz")):
            continue
        rec = st.run(sd, None, max_iter)
        p = W.study_slab(sd)
        np.savez(os.path.join(out_dir, f"layout_{sd:05d}.npz"), donor_map=st.donor_map(p),
                 U=rec["U"].cpu().numpy(), iterations=rec["iterations"], seconds=rec["seconds"],
                 converged=rec["converged"])
        print(json.dumps(dict(seed=sd, iterations=rec["iterations"], seconds=round(rec["seconds"], 3),
                              converged=rec["converged"])), flush=True)


def pack(out_path, sources):
    """Merge converged layouts (per-layout directories written by generate()
    or packed files) into one compressed .npz: seeds, donor_map (int8),
    U (FP32), iterations, seconds.  A seed seen twice keeps its last copy."""
    acc = {}
    for src in sources:
        if os.path.isdir(src):
            for f in sorted(os.listdir(src)):
                if not (f.startswith("layout_") and f.endswith(".npz")):
                    continue
                d = np.load(os.path.join(src, f))
                if bool(d["converged"]):
                    acc[int(f[7:12])] = (d["donor_map"].astype(np.int8), d["U"].astype(np.float32),
                                         int(d["iterations"]), float(d["seconds"]))
        else:
            d = np.load(src)
            for i, sd in enumerate(d["seeds"]):
                acc[int(sd)] = (d["donor_map"][i], d["U"][i], int(d["iterations"][i]), float(d["seconds"][i]))
    keys = sorted(acc)
    np.savez_compressed(out_path, seeds=np.array(keys), donor_map=np.stack([acc[k][0] for k in keys]),
                        U=np.stack([acc[k][1] for k in keys]), iterations=np.array([acc[k][2] for k in keys]),
                        seconds=np.array([acc[k][3] for k in keys]))
    return len(keys)


def load_dataset(data_dir):
    """Converged layouts from a directory of per-layout files, or from one
    packed .npz (arrays seeds, donor_map [n, nz, ny, nx], U [n, nz, ny, nx])."""
    if os.path.isfile(data_dir):
        d = np.load(data_dir)
        return d["donor_map"].astype(np.float32), d["U"].astype(np.float64), [int(v) for v in d["seeds"]]
    xs, us, seeds = [], [], []
    for f in sorted(os.listdir(data_dir)):
        if not f.startswith("layout_") or not f.endswith(".npz"):
            continue
        d = np.load(os.path.join(data_dir, f))
        if not bool(d["converged"]):
            continue
        xs.append(d["donor_map"].astype(np.float32))
        us.append(d["U"].astype(np.float64))
        seeds.append(int(f[7:12]))
    return np.stack(xs), np.stack(us), seeds


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


def near_plane_weights(grid, donor_z, near_weight, half_width=3):
    """Loss weights 1 + near_weight on atom nodes within half_width grid
    planes of the donor plane (where the start error is largest), 1
    elsewhere; float32 [nz, ny, nx]."""
    nx, ny, nz = grid
    m = W.sublattice_masks(W.study_slab(0).pos_q, grid).sum(axis=0) > 0
    z = np.arange(nz)[:, None, None]
    return (1.0 + near_weight * (m & (np.abs(z - donor_z) <= half_width))).astype(np.float32)


def train(data_dir, out_path, epochs=300, lr=1e-3, batch=8, seed=0, target="U", n_val=0, ctx=None,
          dilations=(1, 2, 4, 1), near_weight=0.0):
    """Fit the network to converged potentials.  target "U": the network
    gives U* directly; "E": it gives U* minus the bare-donor potential (the
    electron part), added back at inference.  The targets are taken relative
    to their training mean averaged over the lattice translations (an exact
    symmetry of the donor ensemble), and every epoch shows each layout under
    a random lattice translation.  near_weight > 0 weights the loss on the
    atoms next to the donor plane (near_plane_weights).  The last n_val
    layouts are held out and the max-norm start error on them reported.  The
    learning rate follows a cosine decay from lr to zero."""
    import torch
    st = Study(ctx)
    X, U, seeds = load_dataset(data_dir)
    grid = st.grid
    Ub = np.stack([st.bare_potential(x).cpu().numpy() for x in X])
    feat_scale = float(np.std(Ub))
    Y = U - Ub if target == "E" else U
    ntr = len(X) - n_val
    Tbar = symmetrize(Y[:ntr].mean(axis=0), grid)
    scale = float((Y[:ntr] - Tbar).std())
    T = ((Y - Tbar) / scale).astype(np.float32)
    nz, ny, nx = X.shape[1:]
    net = tbh.Net(st.ctx, (nx, ny, nz), in_channels=N_IN, dilations=dilations)
    net.set_params(W.init_surrogate_weights(seed, in_channels=N_IN, n_layers=len(dilations)))
    if near_weight > 0:
        donor_z = int(np.flatnonzero(X.sum(axis=(0, 2, 3)))[0])
        net.set_loss_weights(torch.from_numpy(near_plane_weights(grid, donor_z, near_weight)).cuda())
    Xd = [st.inputs(x, feat_scale) for x in X]
    Td = [torch.from_numpy(t).cuda() for t in T]
    shifts = lattice_shifts(grid)
    rng = np.random.default_rng(seed)
    Tbar_d = torch.from_numpy(Tbar).cuda()

    def val_errors():
        e = []
        for i in range(ntr, len(X)):
            u = Tbar_d + scale * net.forward(Xd[i]).double()
            if target == "E":
                u = u + torch.from_numpy(Ub[i]).cuda()
            e.append(float((u - torch.from_numpy(U[i]).cuda()).abs().max()))
        return e

    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        lr_ep = 0.5 * lr * (1.0 + np.cos(np.pi * ep / epochs))
        order = rng.permutation(ntr)
        tot = 0.0
        for b0 in range(0, len(order), batch):
            idx = order[b0:b0 + batch]
            xs, ts = [], []
            for i in idx:
                sx, sy = shifts[rng.integers(len(shifts))]
                xs.append(torch.roll(Xd[i], (sy, sx), dims=(2, 3)).contiguous())
                ts.append(torch.roll(Td[i], (sy, sx), dims=(1, 2)).contiguous())
            tot += net.train_step(xs, ts, lr=lr_ep) * len(idx)
        hist.append(tot / len(order))
        if ep % 25 == 0 or ep == epochs - 1:
            rec = dict(epoch=ep, loss=hist[-1], lr=lr_ep)
            if n_val:
                ve = val_errors()
                rec.update(val_err_median=float(np.median(ve)), val_err_max=float(np.max(ve)))
            print(json.dumps(rec), flush=True)
    torch.cuda.synchronize()
    np.savez(out_path, params=net.get_params(), Tbar=Tbar, scale=scale, feat_scale=feat_scale, target=target,
             dilations=np.array(dilations), near_weight=near_weight, loss=np.array(hist),
             train_seeds=np.array(seeds[:ntr]), train_seconds=time.perf_counter() - t0)
    return hist


def evaluate(weights, seeds, max_iter=400, ctx=None, with_mean=True):
    """Per held-out layout: SCF from the zero start, from the mean start (the
    network's output replaced by zero: the symmetrized training mean, plus
    the bare-donor potential for an electron-part model) and from the
    learned start, with the learned start's inference time included."""
    import torch
    st = Study(ctx)
    start = st.surrogate(weights)
    out = []
    for sd in seeds:
        p = W.study_slab(sd)
        dmap = st.donor_map(p)
        zero = st.run(sd, None, max_iter)
        Ustar = zero["U"]
        rec = dict(seed=sd, zero=dict(iterations=zero["iterations"], seconds=zero["seconds"],
                                      converged=zero["converged"]),
                   zero_err0=float(Ustar.abs().max()))
        if with_mean:
            Um = start.Tbar + (st.bare_potential(dmap) if start.target == "E" else 0.0)
            mean = st.run(sd, Um, max_iter, zero["residuals"][0], fallback=True)
            rec["mean"] = dict(iterations=mean["iterations"], seconds=mean["seconds"], converged=mean["converged"],
                               fell_back=mean["fell_back"], err0=float((Um - Ustar).abs().max()))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U0 = start(dmap)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
        learned = st.run(sd, U0, max_iter, zero["residuals"][0], fallback=True)
        rec["learned"] = dict(iterations=learned["iterations"], seconds=learned["seconds"] + t_inf,
                              inference_seconds=t_inf, converged=learned["converged"],
                              fell_back=learned["fell_back"], err0=float((U0 - Ustar).abs().max()),
                              fixed_point_diff=float((learned["U"] - Ustar).abs().max()))
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
    if all("mean" in r for r in records):
        s.update(mean_iters=med("mean", "iterations"), mean_s=med("mean", "seconds"),
                 mean_err0=med("mean", "err0"))
    return s


def main():
    ap = argparse.ArgumentParser()
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
    t.add_argument("--data", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--epochs", type=int, default=300)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--batch", type=int, default=8)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--target", choices=("U", "E"), default="U",
                   help="U: the converged potential; E: its electron part (minus the bare-donor potential)")
    t.add_argument("--val", type=int, default=0, help="hold out this many layouts and report their start error")
    t.add_argument("--dilations", default="1,2,4,1", help="one dilation per layer")
    t.add_argument("--near-weight", type=float, default=0.0,
                   help="extra loss weight on the atoms next to the donor plane")
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--seeds", default="1000:1016")
    e.add_argument("--no-mean", action="store_true", help="skip the mean-start runs")
    e.add_argument("--out", default=None)
    a = ap.parse_args()
    if a.cmd == "gen":
        generate(a.out, _seeds(a.seeds), a.max_iter, a.budget)
    elif a.cmd == "pack":
        print(json.dumps(dict(layouts=pack(a.out, a.sources))), flush=True)
    elif a.cmd == "train":
        train(a.data, a.out, a.epochs, a.lr, a.batch, a.seed, a.target, a.val,
              dilations=tuple(int(v) for v in a.dilations.split(",")), near_weight=a.near_weight)
    else:
        recs = evaluate(a.weights, _seeds(a.seeds), with_mean=not a.no_mean)
        s = summarize(recs)
        print(json.dumps(dict(summary=s)), flush=True)
        if a.out:
            with open(a.out, "w") as f:
                json.dump(dict(records=recs, summary=s), f, indent=1)


if __name__ == "__main__":
    main()
