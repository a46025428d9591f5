"""Train the warm-start network on (delta, u) pairs the solver generates itself,
and measure what it gains as an initial guess.

The solver uses the network on the N/4 mesh: delta there is the mean of 4^3
cells of the N^3 cloud-in-cell density, and the prediction, prolonged twice,
starts the solve at N.  Training pairs are made the same way.  Each pair is a
256^3 solve in a 50 Mpc/h box -- the cell size (100/512 Mpc/h) and particle
mass of the 512^3 mesh of a 100 Mpc/h box -- with the 512^3 workload's
particle recipe: a Zel'dovich lattice (P(k) ~ k^-2, mesh rms 5) plus
Poisson(2.5) Plummer halos of 1e13-1e15 Msun/h (20 per (100 Mpc/h)^3).
|f_R0| is log-uniform in [1e-7, 1e-4], a uniform in [0.5, 1], four draws
per particle load (seeds 10000 + i; held out: 20000 + i); a pair whose solve
does not converge is left out.  The library's cloud-in-cell density and its
mixed-precision solution to relative residual 1e-8 are both restricted to the
64^3 mesh by 4^3 means: the network sees what it sees inside the solver and
learns the restriction of the converged u.  Training: batches of 8 whole 64^3
volumes under random periodic shifts, flips and axis permutations (the field
equation is isotropic), Adam with a cosine learning-rate decay, all forward,
backward and optimiser work in the library's kernels.  Writes the float32
parameter vector (.npy) and a JSON record of the run next to it.

With --evaluate the record also gets V-cycle counts on held-out 512^3 loads
(seeds 20000-20003, a in {0.5, 1}, |f_R0| = 1e-6, the benchmark's schedule)
for four initial guesses: u = 0, the screened-limit guess, the network, and
the best any N/4 prediction could do -- the converged solution itself
restricted to N/4 and interpolated back (trilinear, periodic).

    python -m paper_1305_2418_amd.train_net --pairs 2000 --steps 3000 --evaluate
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np
import torch
import torch.nn.functional as F

from paper_1305_2418_amd import mgfr, synth

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "weights", "unet_warmstart.npy")
FINE = 256                     # mesh and particles per side of one training solve
BOX = 100.0 * FINE / 512       # Mpc/h: the cell size and particle mass of 512^3 in 100 Mpc/h
HALO_RATE = 20.0 * (BOX / 100.0) ** 3
SIDE = FINE // 4               # the network's side (the N/4 mesh)


def _solver(mesh, box, a, fr0, tol=1e-8):
    s = mgfr.Solver(mgfr.Params(mesh=mesh, box=box, a=a, fr0_abs=fr0, tol=tol, precision=mgfr.MIXED,
                                max_vcycles=200, pre_smooth=4, post_smooth=4, coarse_sweeps=30, prolong=1))
    s.set_relaxation32(1.2)
    return s


def make_pairs(n, seed0, per_load=4, log=print):
    """n pairs from ceil(n / per_load) particle loads (seeds seed0 + i), each
    solved at per_load random (a, |f_R0|); pairs whose solve did not converge
    are left out."""
    dev = "cuda"
    rng = np.random.default_rng(seed0)
    D = torch.empty((n, SIDE, SIDE, SIDE), dtype=torch.float32, device=dev)
    Uu = torch.empty_like(D)
    conds = []
    t0 = time.time()
    k = 0
    for i in range((n + per_load - 1) // per_load):
        nh = int(rng.poisson(HALO_RATE))
        pos = synth.clustered_load(FINE, BOX, rms=5.0, seed=seed0 + i, n_halos=nh, device=dev)
        d = None
        for _ in range(min(per_load, n - i * per_load)):
            a = float(rng.uniform(0.5, 1.0))
            fr0 = float(10 ** rng.uniform(-7.0, -4.0))
            s = _solver(FINE, BOX, a, fr0)
            if d is None:
                d = s.assign_density(pos)
            u, _, st = s.solve(d, want_dfr=False, allow_not_converged=True)
            if st.status != 0:
                log(f"load {seed0 + i}: a={a:.3f} |f_R0|={fr0:.2e} stopped at res {st.res:.2e} after "
                    f"{st.vcycles} cycles; left out")
                continue
            D[k] = F.avg_pool3d(d[None, None], 4)[0, 0].float()
            Uu[k] = F.avg_pool3d(u[None, None], 4)[0, 0].float()
            conds.append((a, fr0))
            k += 1
            del s, u
        del pos, d
        if (i + 1) % 25 == 0:
            log(f"loads {i + 1}, pairs {k}/{n} ({time.time() - t0:.0f}s)")
    return D[:k], Uu[:k], conds


def augment(d, u, gen):
    """The same random periodic shift, axis flips and axis permutation of both volumes."""
    sh = torch.randint(0, d.shape[0], (3,), generator=gen).tolist()
    d, u = torch.roll(d, sh, (0, 1, 2)), torch.roll(u, sh, (0, 1, 2))
    flips = [ax for ax in range(3) if torch.rand((), generator=gen).item() < 0.5]
    if flips:
        d, u = torch.flip(d, flips), torch.flip(u, flips)
    perm = torch.randperm(3, generator=gen).tolist()
    return d.permute(perm), u.permute(perm)


def batch(D, Uu, conds, idx, gen):
    ds, us = zip(*(augment(D[i], Uu[i], gen) for i in idx))
    return (torch.stack(ds).double().contiguous(), torch.stack(us).double().contiguous(), [conds[i] for i in idx])


def _prolong_trilinear(c, f):
    """Periodic trilinear interpolation of a cell-centred field by a factor f."""
    S = c.shape[0]
    x = F.pad(c[None, None], (1, 1, 1, 1, 1, 1), mode="circular")
    y = F.interpolate(x, scale_factor=f, mode="trilinear", align_corners=False)
    return y[0, 0, f:f + S * f, f:f + S * f, f:f + S * f].contiguous()


def evaluate(net, seeds=(20000, 20001, 20002, 20003), scale_factors=(0.5, 1.0), fr0=1e-6, log=print):
    """V-cycles and solve times from four initial guesses on held-out 512^3 loads."""
    dev, N = "cuda", 512
    rows = []
    for seed in seeds:
        pos = synth.clustered_load(N, 100.0, rms=5.0, seed=seed, n_halos=20, device=dev)
        for a in scale_factors:
            s = _solver(N, 100.0, a, fr0)
            snn = mgfr.Solver(mgfr.Params(mesh=N, box=100.0, a=a, fr0_abs=fr0, tol=1e-8, precision=mgfr.MIXED,
                                          max_vcycles=200, pre_smooth=4, post_smooth=4, coarse_sweeps=30,
                                          prolong=1, nn_mode=mgfr.NN_COARSE))
            snn.set_relaxation32(1.2)
            snn.set_net(net)
            d = s.assign_density(pos)
            ustar, _, _ = _solver(N, 100.0, a, fr0, tol=1e-11).solve(d, want_dfr=False)
            guesses = {"cold": None, "screened": s.screened_guess(d),
                       "ideal N/4": _prolong_trilinear(F.avg_pool3d(ustar[None, None], 4)[0, 0], 4)}
            row = {"seed": seed, "a": a, "fr0": fr0}
            for name, g in guesses.items():
                torch.cuda.synchronize()
                t = time.perf_counter()
                _, _, st = s.solve(d, u=None if g is None else g.clone(), want_dfr=False)
                torch.cuda.synchronize()
                row[name] = {"vcycles": st.vcycles, "res0": st.res0, "ms": 1e3 * (time.perf_counter() - t)}
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, _, st = snn.solve(d, want_dfr=False)
            torch.cuda.synchronize()
            row["network"] = {"vcycles": st.vcycles, "res0": st.res0, "ms": 1e3 * (time.perf_counter() - t)}
            rows.append(row)
            log(f"seed {seed} a={a}: " + ", ".join(f"{k} {row[k]['vcycles']}" for k in
                                                   ("cold", "screened", "network", "ideal N/4")))
            del s, snn, d, ustar, guesses
        del pos
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--evaluate", action="store_true", help="also time solves on held-out 512^3 loads")
    ap.add_argument("--evaluate-only", action="store_true", help="evaluate the weights at --out, no training")
    args = ap.parse_args()
    log = lambda m: print(m, flush=True)
    meta_path = os.path.splitext(args.out)[0] + ".json"
    if args.evaluate_only:
        net = mgfr.Net(seed=0, max_voxels=128 ** 3)
        net.set_params(np.load(args.out))
        meta = json.load(open(meta_path)) if os.path.exists(meta_path) else {}
        meta["evaluation"] = evaluate(net, log=log)
        json.dump(meta, open(meta_path, "w"), indent=1)
        return
    t0 = time.time()
    D, Uu, conds = make_pairs(args.pairs, 10000, log=log)
    t_pairs = time.time() - t0
    log(f"generated {D.shape[0]} pairs in {t_pairs:.0f}s")
    Dv, Uv, cv = make_pairs(8, 20000, log=log)
    net = mgfr.Net(seed=args.seed, max_voxels=max(args.batch * SIDE ** 3, 128 ** 3))
    gen = torch.Generator().manual_seed(args.seed)
    curve = []
    t1 = time.time()
    for it in range(args.steps):
        lr = 1e-4 + 0.5 * (args.lr - 1e-4) * (1 + math.cos(math.pi * it / args.steps))
        idx = torch.randint(0, D.shape[0], (args.batch,), generator=gen).tolist()
        d, u, c = batch(D, Uu, conds, idx, gen)
        L = net.train_step(d, u, c, lr)
        if it % 50 == 0 or it == args.steps - 1:
            curve.append((it, L))
            log(f"step {it} loss {L:.5f} lr {lr:.2e} ({time.time() - t1:.0f}s)")
    t_train = time.time() - t1
    held = []
    for i in range(Dv.shape[0]):
        pred = net.predict(Dv[i:i + 1].double().contiguous(), [cv[i]])
        held.append((((pred - Uv[i:i + 1].double()) / 5.0) ** 2).mean().item())
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    np.save(args.out, net.get_params())
    meta = {"pairs": int(D.shape[0]), "loads": (args.pairs + 3) // 4, "fine_mesh": FINE, "box": BOX, "side": SIDE, "batch": args.batch,
            "steps": args.steps, "lr": args.lr, "seed": args.seed, "t_pairs_s": t_pairs, "t_train_s": t_train,
            "loss_curve": curve, "heldout_loss": held,
            "recipe": f"{FINE}^3 particles and mesh in {BOX:g} Mpc/h (the 512^3-in-100 Mpc/h cell), Zel'dovich "
                      f"k^-2 rms 5 + Poisson({HALO_RATE:g}) Plummer halos 1e13-1e15, |f_R0| log-U[1e-7,1e-4], "
                      "a U[0.5,1] (four draws per load), delta and converged u restricted to 64^3 by 4^3 means, seeds 10000+i "
                      "(held out 20000+i)"}
    if args.evaluate:
        del D, Uu
        meta["evaluation"] = evaluate(net, log=log)
    json.dump(meta, open(meta_path, "w"), indent=1)
    log(f"saved {args.out}; held-out loss {np.mean(held):.5f}")


if __name__ == "__main__":
    main()
