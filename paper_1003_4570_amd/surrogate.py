"""Learned start potential for the self-consistent loop.

    python -m paper_1003_4570_amd.surrogate gen   --out DIR --seeds 0:96
    python -m paper_1003_4570_amd.surrogate train --data DIR --out W.npz
    python -m paper_1003_4570_amd.surrogate eval  --weights W.npz --seeds 1000:1016

The self-consistent Schrodinger-Poisson loop (Sec. III-A) is run by the
library (tbh_scf_*); this module drives it: it generates converged
potentials with the plain method (zero start, linear mixing), trains the
convolutional surrogate on them with the library's device kernels
(tbh_net_*), and compares SCF time-to-converge from the zero start, the
training-mean start and the learned start on held-out donor layouts.  The
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


def train(data_dir, out_path, epochs=300, lr=1e-3, batch=8, seed=0, ctx=None):
    import torch
    ctx = ctx or tbh.Context(0)
    X, U, seeds = load_dataset(data_dir)
    Ubar = U.mean(axis=0)
    scale = float((U - Ubar).std())
    T = ((U - Ubar) / scale).astype(np.float32)
    nz, ny, nx = X.shape[1:]
    net = tbh.Net(ctx, (nx, ny, nz))
    net.set_params(W.init_surrogate_weights(seed))
    Xd = [torch.from_numpy(x).cuda() for x in X]
    Td = [torch.from_numpy(t).cuda() for t in T]
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(Xd))
        tot = 0.0
        for b0 in range(0, len(order), batch):
            idx = order[b0:b0 + batch]
            tot += net.train_step([Xd[i] for i in idx], [Td[i] for i in idx], lr=lr) * len(idx)
        hist.append(tot / len(order))
        if ep % 25 == 0 or ep == epochs - 1:
            print(json.dumps(dict(epoch=ep, loss=hist[-1])), flush=True)
    torch.cuda.synchronize()
    np.savez(out_path, params=net.get_params(), Ubar=Ubar, scale=scale, loss=np.array(hist),
             train_seeds=np.array(seeds), train_seconds=time.perf_counter() - t0)
    return hist


def learned_start(net, Ubar, scale, donor_map):
    import torch
    y = net.forward(torch.from_numpy(donor_map.astype(np.float32)).cuda())
    return torch.from_numpy(Ubar).cuda() + scale * y.double()


def evaluate(weights, seeds, max_iter=400, ctx=None):
    import torch
    st = Study(ctx)
    wz = np.load(weights)
    nz, ny, nx = wz["Ubar"].shape
    net = tbh.Net(st.ctx, (nx, ny, nz))
    net.set_params(wz["params"])
    Ubar = wz["Ubar"]
    scale = float(wz["scale"])
    out = []
    for sd in seeds:
        p = W.study_slab(sd)
        zero = st.run(sd, None, max_iter)
        Ustar = zero["U"]
        mean = st.run(sd, torch.from_numpy(Ubar).cuda(), max_iter, zero["residuals"][0], fallback=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U0 = learned_start(net, Ubar, scale, st.donor_map(p))
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
        learned = st.run(sd, U0, max_iter, zero["residuals"][0], fallback=True)
        rec = dict(seed=sd,
                   zero=dict(iterations=zero["iterations"], seconds=zero["seconds"], converged=zero["converged"]),
                   mean=dict(iterations=mean["iterations"], seconds=mean["seconds"], converged=mean["converged"],
                             fell_back=mean["fell_back"],
                             err0=float((torch.from_numpy(Ubar).cuda() - Ustar).abs().max())),
                   learned=dict(iterations=learned["iterations"], seconds=learned["seconds"] + t_inf,
                                inference_seconds=t_inf, converged=learned["converged"],
                                fell_back=learned["fell_back"], err0=float((U0 - Ustar).abs().max()),
                                fixed_point_diff=float((learned["U"] - Ustar).abs().max())),
                   zero_err0=float(Ustar.abs().max()))
        out.append(rec)
        print(json.dumps(rec), flush=True)
    return out


def summarize(records):
    def med(key, sub):
        return float(np.median([r[key][sub] for r in records]))
    return dict(n=len(records), zero_iters=med("zero", "iterations"), mean_iters=med("mean", "iterations"),
                learned_iters=med("learned", "iterations"), zero_s=med("zero", "seconds"),
                mean_s=med("mean", "seconds"), learned_s=med("learned", "seconds"),
                speedup_time=med("zero", "seconds") / med("learned", "seconds"),
                speedup_iters=med("zero", "iterations") / med("learned", "iterations"),
                learned_err0=med("learned", "err0"), mean_err0=med("mean", "err0"),
                zero_err0=float(np.median([r["zero_err0"] for r in records])),
                fallbacks=int(sum(r["learned"]["fell_back"] for r in records)))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    g = sub.add_parser("gen")
    g.add_argument("--out", required=True)
    g.add_argument("--seeds", default="0:96")
    g.add_argument("--max-iter", type=int, default=400)
    g.add_argument("--budget", type=float, default=None, help="stop starting layouts after this many seconds")
    t = sub.add_parser("train")
    t.add_argument("--data", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--epochs", type=int, default=300)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--batch", type=int, default=8)
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--seeds", default="1000:1016")
    e.add_argument("--out", default=None)
    a = ap.parse_args()
    if a.cmd == "gen":
        generate(a.out, _seeds(a.seeds), a.max_iter, a.budget)
    elif a.cmd == "train":
        train(a.data, a.out, a.epochs, a.lr, a.batch)
    else:
        recs = evaluate(a.weights, _seeds(a.seeds))
        s = summarize(recs)
        print(json.dumps(dict(summary=s)), flush=True)
        if a.out:
            with open(a.out, "w") as f:
                json.dump(dict(records=recs, summary=s), f, indent=1)


if __name__ == "__main__":
    main()
