"""Throughput of the f(R) hot path on one MI355X.

One step = cloud-in-cell assignment of the particles, the FAS multigrid solve
from a cold start (u = 0) to relative residual 1e-8, and the fifth force
gathered back to every particle, on a synthetic clustered particle load that
is resident in HBM before the timed region.  Prints one JSON line.

Default workload: 512^3 particles (float32 positions) on a 512^3 mesh,
100 Mpc/h box, a = 1, |f_R0| = 1e-6, Zel'dovich lattice with P(k) ~ k^-2
(rms 5) plus 20 Plummer halos of 1e13-1e15 Msun/h.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mesh", type=int, default=512)
    ap.add_argument("--a", type=float, default=1.0)
    ap.add_argument("--fr0", type=float, default=1e-6)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--mode", choices=["fp64", "mixed", "mixed_nn"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-mesh", type=int, default=128)
    return ap.parse_args()


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


SWEEP_SRC = ["paper_1305_2418_amd/csrc/mgfr_solver.hip"]


def cpu_baseline(args, log):
    """The FP64 oracle, as it stands, on a bounded sample of the same recipe."""
    import numpy as np
    from oracle import oracle as O
    from paper_1305_2418_amd import synth
    N = args.cpu_mesh
    pos = synth.clustered_load(N, 100.0, rms=5.0, seed=args.seed, n_halos=20).numpy()
    t0 = time.perf_counter()
    m = O.cic_assign(N, 100.0, pos)
    d = O.density_contrast(m)
    p = O.params(mesh=N, a=args.a, fr0_abs=args.fr0, tol=1e-8)
    s, u, dfr, st = O.solve(p, d)
    acc = O.fifth_force(p, u, pos)
    dt = time.perf_counter() - t0
    log(f"cpu oracle {N}^3: {dt:.2f}s, {st.vcycles} V-cycles, status {s}")
    return {"value": N ** 3 / dt, "unit": "cells/s", "cores": 1, "kind": "oracle",
            "sample": f"{N}^3 mesh and {N}^3 particles of the same recipe (seed {args.seed}), "
                      f"one full step (CIC + FP64 FAS solve to 1e-8 + fifth force), "
                      f"{st.vcycles} V-cycles, single-threaded C oracle, {os.cpu_count()} host cpus seen"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    import torch
    from paper_1305_2418_amd import mgfr, synth

    dev = torch.device("cuda:0")
    N = args.mesh
    t0 = time.perf_counter()
    pos = synth.clustered_load(N, 100.0, rms=5.0, seed=args.seed, n_halos=20, device=dev).to(dev)
    torch.cuda.synchronize()
    log(f"generated {N}^3 particles in {time.perf_counter() - t0:.1f}s")

    precision = mgfr.MIXED if args.mode in ("mixed", "mixed_nn") else mgfr.FP64
    nn_mode = mgfr.NN_COARSE if args.mode == "mixed_nn" else mgfr.NN_NONE
    params = mgfr.Params(mesh=N, box=100.0, a=args.a, fr0_abs=args.fr0, tol=1e-8,
                         precision=precision, nn_mode=nn_mode, max_vcycles=100)
    solver = mgfr.Solver(params)
    delta = torch.empty((N, N, N), dtype=torch.float64, device=dev)
    u = torch.zeros_like(delta)
    acc = torch.empty((pos.shape[0], 3), dtype=torch.float32, device=dev)

    def step(timing=False):
        solver.set_timing(timing)
        solver.assign_density(pos, out=delta)
        u.zero_()
        _, dfr, st = solver.solve(delta, u=u, want_dfr=True)
        solver.fifth_force(u, pos, out=acc)
        return st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = 1e3 * elapsed / args.steps

    # separate pass with per-launch HIP events on the finest-level smoothing kernel
    st_t = step(timing=True)
    torch.cuda.synchronize()
    sweep_ms = st_t.t_sweep_ms / max(1, st_t.n_sweep_launches)
    # algorithmic bytes of one full red-black sweep of the finest level: read u and f,
    # write u = 24 B per cell (one fused launch at N >= 512, two per-colour launches below)
    alg_bytes = 24.0 * N ** 3
    kernel = "k_sweep_fused" if N >= 512 else "k_sweep_half (x2 per sweep)"
    achieved = alg_bytes / (sweep_ms * 1e-3) / 1e9
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "sweep_traffic.json")
    if os.path.exists(tpath):
        tj = json.load(open(tpath))
        if tj.get("source_hash") == source_hash(SWEEP_SRC) and tj.get("mesh") == N:
            traffic = tj.get("bytes_per_launch")
    solve_ms = sum(s.t_solve_ms for s in stats) / len(stats)
    vcyc = [s.vcycles for s in stats]
    log(f"step {ms:.2f} ms, solve {solve_ms:.2f} ms, V-cycles {vcyc}, res {stats[-1].res:.2e}, "
        f"sweep launch {sweep_ms:.3f} ms ({achieved:.0f} GB/s algorithmic)")

    out = {
        "metric": "cells/s to converged f_R solve (res<1e-8), plain FP64 MG vs mixed+NN warm start",
        "value": N ** 3 / (ms * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == mgfr.FP64 else "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": f"{N}^3 mesh, {N}^3 particles, 100 Mpc/h, a={args.a}, |f_R0|={args.fr0}, "
                        f"Zel'dovich k^-2 rms 5 + 20 Plummer halos, seed {args.seed}; step = CIC + "
                        f"solve from u=0 to 1e-8 + fifth force",
            "mode": args.mode,
            "solve_ms": solve_ms,
            "solve_cells_per_s": N ** 3 / (solve_ms * 1e-3),
            "vcycles": vcyc,
            "res": stats[-1].res,
        },
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel, "launch_ms": sweep_ms,
                     "alg_bytes_per_launch": alg_bytes},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
