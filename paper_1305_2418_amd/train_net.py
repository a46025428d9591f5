"""Train the warm-start network on (delta, u) pairs the solver generates itself.

Pairs: 128^3 meshes of a 100 Mpc/h box with the 512^3 workload's particle
recipe at 128^3 (Zel'dovich lattice, P(k) ~ k^-2, rms 5, plus 20 Plummer
halos of 1e13-1e15 Msun/h); |f_R0| log-uniform in [1e-7, 1e-4], a uniform in
[0.5, 1]; seeds 10000 + i.  Each delta is the cloud-in-cell density of the
library, each target the library's mixed-precision solution to relative
residual 1e-8.  Training: random periodic 64^3 crops, batch 8, Adam with a
cosine learning-rate decay, all forward/backward/optimiser work in the
library's kernels.  Writes the float32 parameter vector (.npy) and a JSON
record of the run next to it.

    python -m paper_1305_2418_amd.train_net --pairs 2000 --steps 3000
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np
import torch

from paper_1305_2418_amd import mgfr, synth

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "weights", "unet_warmstart.npy")


def make_pairs(n, side, seed0, box=100.0, log=print):
    dev = "cuda"
    rng = np.random.default_rng(seed0)
    D = torch.empty((n, side, side, side), dtype=torch.float32, device=dev)
    Uu = torch.empty_like(D)
    conds = []
    solvers = {}
    t0 = time.time()
    for i in range(n):
        a = float(rng.uniform(0.5, 1.0))
        fr0 = float(10 ** rng.uniform(-7.0, -4.0))
        pos = synth.clustered_load(side, box, rms=5.0, seed=seed0 + i, n_halos=20, device=dev)
        s = mgfr.Solver(mgfr.Params(mesh=side, box=box, a=a, fr0_abs=fr0, precision=mgfr.MIXED, max_vcycles=200))
        d = s.assign_density(pos)
        u, _, st = s.solve(d, want_dfr=False, allow_not_converged=True)
        if st.status != 0:
            log(f"pair {seed0 + i}: a={a:.3f} |f_R0|={fr0:.2e} stopped at res {st.res:.2e} after {st.vcycles} cycles")
        D[i] = d.float()
        Uu[i] = u.float()
        conds.append((a, fr0))
        if (i + 1) % 100 == 0:
            log(f"pairs {i + 1}/{n} ({time.time() - t0:.0f}s)")
    return D, Uu, conds


def crops(D, Uu, conds, idx, crop, gen):
    side = D.shape[1]
    ds, us, cs = [], [], []
    for i in idx:
        sh = torch.randint(0, side, (3,), generator=gen).tolist()
        d = torch.roll(D[i], shifts=sh, dims=(0, 1, 2))[:crop, :crop, :crop]
        u = torch.roll(Uu[i], shifts=sh, dims=(0, 1, 2))[:crop, :crop, :crop]
        ds.append(d)
        us.append(u)
        cs.append(conds[i])
    return torch.stack(ds).double().contiguous(), torch.stack(us).double().contiguous(), cs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--side", type=int, default=128)
    ap.add_argument("--crop", type=int, default=64)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_OUT)
    args = ap.parse_args()
    log = lambda m: print(m, flush=True)
    t0 = time.time()
    D, Uu, conds = make_pairs(args.pairs, args.side, 10000, log=log)
    t_pairs = time.time() - t0
    log(f"generated {args.pairs} pairs in {t_pairs:.0f}s")
    Dv, Uv, cv = make_pairs(4, args.side, 20000, log=log)
    net = mgfr.Net(seed=args.seed, max_voxels=max(args.batch * args.crop ** 3, args.side ** 3))
    gen = torch.Generator().manual_seed(args.seed)
    curve = []
    t1 = time.time()
    for it in range(args.steps):
        lr = 1e-4 + 0.5 * (args.lr - 1e-4) * (1 + math.cos(math.pi * it / args.steps))
        idx = torch.randint(0, args.pairs, (args.batch,), generator=gen).tolist()
        d, u, c = crops(D, Uu, conds, idx, args.crop, gen)
        L = net.train_step(d, u, c, lr)
        if it % 50 == 0 or it == args.steps - 1:
            curve.append((it, L))
            log(f"step {it} loss {L:.5f} lr {lr:.2e} ({time.time() - t1:.0f}s)")
    t_train = time.time() - t1
    # held-out loss on full 128^3 volumes
    held = []
    for i in range(Dv.shape[0]):
        pred = net.predict(Dv[i:i + 1].double().contiguous(), [cv[i]])
        err = ((pred - Uv[i:i + 1].double()) / 5.0) ** 2
        held.append(err.mean().item())
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out, net.get_params())
    meta = {"pairs": args.pairs, "side": args.side, "crop": args.crop, "batch": args.batch, "steps": args.steps,
            "lr": args.lr, "seed": args.seed, "t_pairs_s": t_pairs, "t_train_s": t_train,
            "loss_curve": curve, "heldout_loss": held,
            "recipe": "100 Mpc/h, 128^3 particles, Zel'dovich k^-2 rms 5 + 20 Plummer halos 1e13-1e15, "
                      "|f_R0| log-U[1e-7,1e-4], a U[0.5,1], seeds 10000+i (held out 20000+i)"}
    json.dump(meta, open(os.path.splitext(args.out)[0] + ".json", "w"), indent=1)
    log(f"saved {args.out}; held-out loss {np.mean(held):.5f}")


if __name__ == "__main__":
    main()
