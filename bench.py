"""Throughput of the f(R) hot path on one MI355X.

One step = cloud-in-cell assignment of the particles, the FAS multigrid solve
from a cold start to relative residual 1e-8, and the fifth force gathered
back to every particle, on a synthetic clustered particle load that is
resident in HBM before the timed region.  Prints one JSON line.

Default workload: 512^3 particles (float32 positions) on a 512^3 mesh,
100 Mpc/h box, a = 1, |f_R0| = 1e-6, Zel'dovich lattice with P(k) ~ k^-2
(rms 5) plus 20 Plummer halos of 1e13-1e15 Msun/h, V(4,4) cycles with the
correction injected into the daughter cells.  The
headline mode is the mixed-precision solve with the learned warm start;
the plain float64 solve and the mixed solve without the network are timed
in the same run on the same input and reported beside it.
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
WEIGHTS = os.path.join(ROOT, "paper_1305_2418_amd", "weights", "unet_warmstart.npy")
MODES = ("fp64", "mixed", "mixed_nn", "mixed_scr", "fp64_scr")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mesh", type=int, default=512)
    ap.add_argument("--a", type=float, default=1.0)
    ap.add_argument("--fr0", type=float, default=1e-6)
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--smooth", type=int, default=4, help="pre- and post-smoothing sweeps")
    ap.add_argument("--omega", type=float, default=1.2,
                    help="relaxation factor of the float32 correction sweeps of the mixed modes (1: plain NGS)")
    ap.add_argument("--inner", type=int, default=3,
                    help="float32 correction V-cycles per float64 residual check of the mixed modes, at most")
    ap.add_argument("--coarse-sweeps", type=int, default=None,
                    help="red-black sweeps on the coarsest grid (default: 30 for the uniform mesh, whose 4^3 "
                         "level runs inside one launch; 4 for the adaptive workload, whose refined levels' "
                         "coarsest sublevel costs a launch per colour and sweep)")
    ap.add_argument("--prolong", choices=["inject", "linear"], default="inject",
                    help="coarse-to-fine transfer of the correction (both are the paper's options)")
    ap.add_argument("--mode", choices=MODES, default="mixed_nn", help="headline mode")
    ap.add_argument("--compare", default="fp64,mixed,mixed_scr",
                    help="other modes timed in the same run (_scr: from the screened-limit initial guess)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["uniform", "amr", "sequence"], default="uniform",
                    help="amr: 256^3 base + 2 block-refined levels on 256^3 particles with 50 NFW halos; "
                         "sequence: consecutive steps of a growing displacement field, each solve warm-started "
                         "in several ways")
    ap.add_argument("--also-a", default="0.5",
                    help="comma-separated other scale factors at which mixed, mixed_nn and mixed_scr are also timed")
    ap.add_argument("--no-fixed-compare", action="store_true",
                    help="amr workload: skip the untimed adaptive-versus-fixed spectra (profiling the step alone)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also stream 1 GiB through a plain elementwise kernel (reference for HBM counters)")
    return ap.parse_args()


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


# sources of the timed sweep kernels (a traffic record applies only to the code it was counted on)
KERNEL_SRC = {"fp64": ["paper_1305_2418_amd/csrc/mgfr_solver.hip", "paper_1305_2418_amd/csrc/mgfr_ops.h"],
              "mixed": ["paper_1305_2418_amd/csrc/mgfr_mixed.hip", "paper_1305_2418_amd/csrc/mgfr_ops.h"]}


def prolong_code(args):
    return 1 if args.prolong == "inject" else 0


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, log):
    """The FP64 oracle, as it stands, on a bounded sample of the same recipe:
    its OpenMP build on the host's threads at N/2 (the headline figure) and
    its single-thread build at N/4.  Also returns the N/2 sample and the
    oracle's solution of it iterated to 1e-11, for the error of the library's
    mixed solve against the oracle."""
    from oracle import oracle as O
    from paper_1305_2418_amd import synth
    threads = O.threads()
    res = {}
    for tag, N, serial in (("omp", args.mesh // 2, False), ("serial", args.mesh // 4, True)):
        pos = synth.clustered_load(N, 100.0, rms=5.0, seed=args.seed, n_halos=20).numpy()
        t0 = time.perf_counter()
        m = O.cic_assign(N, 100.0, pos, serial=serial)
        d = O.density_contrast(m, serial=serial)
        p = O.params(mesh=N, a=args.a, fr0_abs=args.fr0, tol=1e-8, pre_smooth=args.smooth,
                     post_smooth=args.smooth, prolong=prolong_code(args))
        s, u, dfr, st = O.solve(p, d, serial=serial)
        O.fifth_force(p, u, pos, serial=serial)
        dt = time.perf_counter() - t0
        log(f"cpu oracle ({tag}, {1 if serial else threads} threads) {N}^3: {dt:.2f}s, {st.vcycles} V-cycles")
        res[tag] = dict(N=N, dt=dt, cycles=st.vcycles, delta=d, u=u, p=p)
    o = res["omp"]
    pt = O.params(mesh=o["N"], a=args.a, fr0_abs=args.fr0, tol=1e-11, pre_smooth=args.smooth,
                  post_smooth=args.smooth, prolong=prolong_code(args))
    _, _, dfr_tight, _ = O.solve(pt, o["delta"], u0=o["u"])
    sr = res["serial"]
    base = {"value": o["N"] ** 3 / o["dt"], "unit": "cells/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus_seen": os.cpu_count(),
            "sample": f"{o['N']}^3 mesh and {o['N']}^3 particles of the same recipe (seed {args.seed}), one full "
                      f"step (CIC + FP64 FAS V({args.smooth},{args.smooth}) {args.prolong} solve to 1e-8 + fifth "
                      f"force), OpenMP build of the C oracle on {threads} threads",
            "oracle_vcycles": o["cycles"],
            "single_thread": {"value": sr["N"] ** 3 / sr["dt"], "unit": "cells/s", "cores": 1,
                              "sample": f"{sr['N']}^3 of the same recipe", "oracle_vcycles": sr["cycles"]}}
    return base, o["delta"], dfr_tight


def mixed_vs_oracle(args, delta, dfr_oracle, dev, log):
    """The library's mixed solve (headline schedule and omega) of the oracle's
    sample: max-norm relative delta f_R difference from the oracle's solution."""
    import torch
    from paper_1305_2418_amd import mgfr
    N = delta.shape[0]
    s = mgfr.Solver(mgfr.Params(mesh=N, box=100.0, a=args.a, fr0_abs=args.fr0, tol=1e-8, precision=mgfr.MIXED,
                                pre_smooth=args.smooth, post_smooth=args.smooth, prolong=prolong_code(args)))
    s.set_relaxation32(args.omega)
    s.set_inner_cycles(args.inner)
    u, dfr, st = s.solve(torch.tensor(delta, device=dev))
    ref = torch.tensor(dfr_oracle, device=dev)
    err = float((dfr - ref).abs().max() / ref.abs().max())
    log(f"mixed solve of the {N}^3 oracle sample: {st.vcycles} cycles, rel dfr difference from the oracle {err:.2e}")
    return {"mesh": N, "rel_dfr_vs_oracle": err, "vcycles": st.vcycles, "oracle_tol": 1e-11}


# The network's convolutions (input channels, output channels, level: 0 = S, 1 = S/2, 2 = S/4)
NET_CONVS = [(16, 16, 0), (16, 16, 0), (16, 32, 1), (32, 32, 1), (32, 64, 2), (64, 64, 2),
             (96, 32, 1), (32, 32, 1), (48, 16, 0), (16, 16, 0)]


def net_forward_flops(S):
    return sum(2 * 27 * ci * co * (S >> lev) ** 3 for ci, co, lev in NET_CONVS)


def measure_mfma(N, dev, log):
    """The network's forward pass on the N/4 mesh (its use in the warm start) timed with HIP events."""
    import numpy as np
    import torch
    from paper_1305_2418_amd import mgfr
    S = N // 4
    net = mgfr.Net(seed=0, max_voxels=S ** 3)
    net.set_params(np.load(WEIGHTS))
    d = torch.randn((1, S, S, S), dtype=torch.float64, generator=torch.Generator().manual_seed(1)).to(dev)
    cond = [(1.0, 1e-6)]
    for _ in range(2):
        net.predict(d, cond)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    a.record()
    for _ in range(reps):
        net.predict(d, cond)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    tf = net_forward_flops(S) / (ms * 1e-3) / 1e12
    log(f"network forward at {S}^3: {ms:.3f} ms, {tf:.1f} TFLOP/s")
    return {"kernel": f"k_conv3d (network forward, {S}^3, bf16 MFMA 16x16x32)", "ms": ms,
            "flop": net_forward_flops(S), "achieved": tf, "peak": 2500.0, "unit": "TFLOP/s",
            "frac": tf / 2500.0}


def measure_copy(dev, log):
    """Achievable streaming bandwidth: bitwise NOT of 1 GiB into a second buffer, HIP events."""
    import torch
    n = 1 << 28
    x = torch.ones(n, dtype=torch.int32, device=dev)
    y = torch.empty_like(x)
    for _ in range(2):
        torch.bitwise_not(x, out=y)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    a.record()
    for _ in range(reps):
        torch.bitwise_not(x, out=y)
    b.record()
    torch.cuda.synchronize()
    gbs = 2.0 * (1 << 30) * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    log(f"streaming kernel: {gbs:.0f} GB/s")
    del x, y
    return gbs


def run_mode(mode, args, pos, dev, log, a=None, dfr_ref=None):
    import numpy as np
    import torch
    from paper_1305_2418_amd import mgfr
    N = args.mesh
    a = args.a if a is None else a
    precision = mgfr.FP64 if mode.startswith("fp64") else mgfr.MIXED
    screened = mode.endswith("_scr")
    nn_mode = mgfr.NN_COARSE if mode == "mixed_nn" else mgfr.NN_NONE
    params = mgfr.Params(mesh=N, box=100.0, a=a, fr0_abs=args.fr0, tol=1e-8, precision=precision,
                         nn_mode=nn_mode, max_vcycles=100, pre_smooth=args.smooth, post_smooth=args.smooth,
                         coarse_sweeps=30 if args.coarse_sweeps is None else args.coarse_sweeps,
                         prolong=prolong_code(args))
    solver = mgfr.Solver(params)
    if precision == mgfr.MIXED:
        solver.set_relaxation32(args.omega)
        solver.set_inner_cycles(args.inner)
    net = None
    if nn_mode == mgfr.NN_COARSE:
        if not os.path.exists(WEIGHTS):
            raise SystemExit(f"{WEIGHTS} missing: train it with python -m paper_1305_2418_amd.train_net")
        net = mgfr.Net(seed=0, max_voxels=(N // 4) ** 3)
        net.set_params(np.load(WEIGHTS))
        solver.set_net(net)
    delta = torch.empty((N, N, N), dtype=torch.float64, device=dev)
    u = torch.zeros_like(delta)
    acc = torch.empty((pos.shape[0], 3), dtype=torch.float32, device=dev)

    last = {}

    def step(timing=False):
        solver.set_timing(timing)
        solver.assign_density(pos, out=delta)
        if screened:
            solver.screened_guess(delta, out=u)
        elif nn_mode != mgfr.NN_COARSE:  # the network's guess overwrites u
            u.zero_()
        _, dfr, st = solver.solve(delta, u=u, want_dfr=True)
        solver.fifth_force(u, pos, out=acc)
        last["dfr"] = dfr
        return st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(step())
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    # separate pass with per-launch HIP events around the finest-level smoothing kernel
    st_t = step(timing=True)
    torch.cuda.synchronize()
    sweep_ms = st_t.t_sweep_ms / max(1, st_t.n_sweep_launches)
    solve_ms = sum(s.t_solve_ms for s in stats) / len(stats)
    out = {"ms_per_step": ms, "solve_ms": solve_ms, "cells_per_s": N ** 3 / (ms * 1e-3),
           "solve_cells_per_s": N ** 3 / (solve_ms * 1e-3), "vcycles": [s.vcycles for s in stats],
           "res": stats[-1].res, "fell_back": max(s.fell_back for s in stats), "nn_ms": stats[-1].t_nn_ms,
           "sweep_launch_ms": sweep_ms, "dfr_max": float(last["dfr"].abs().max())}
    if dfr_ref is not None:
        # max-norm relative difference of delta f_R from the float64 solve of the same input
        out["rel_dfr_vs_fp64"] = float((last["dfr"] - dfr_ref).abs().max() / dfr_ref.abs().max())
        log(f"[{mode} a={a}] max-norm relative delta f_R difference from the float64 solve: "
            f"{out['rel_dfr_vs_fp64']:.2e}")
    if mode == "fp64":
        out["_dfr"] = last["dfr"]
    log(f"[{mode} a={a}] step {ms:.2f} ms, solve {solve_ms:.2f} ms, V-cycles {out['vcycles']}, res {out['res']:.2e}, "
        f"sweep launch {sweep_ms:.3f} ms, nn {out['nn_ms']:.2f} ms")
    if mode == args.mode and a == args.a:
        # the power-spectrum diagnostic of the last solution (untimed): P(delta + delta_eff) / P(delta)
        k, ratio, _, _ = solver.power_ratio(delta, solver.effective_density(delta, u))
        sel = list(range(0, len(k), max(1, len(k) // 16)))
        out["power_ratio"] = {"k_h_per_Mpc": [float(k[i]) for i in sel], "ratio": [float(ratio[i]) for i in sel]}
        log("[power ratio] " + ", ".join(f"k={k[i]:.2f}: {ratio[i]:.3f}" for i in sel[::4]))
    del solver, net
    return out


def run_amr(args, log):
    """Adaptive workload: base solve plus two refined levels per step."""
    import torch
    from paper_1305_2418_amd import mgfr, synth
    N0 = 256
    dev = torch.device("cuda:0")
    pos = synth.clustered_load(N0, 100.0, rms=5.0, seed=4, n_halos=50, profile="nfw", device=dev).to(dev)
    params = mgfr.Params(mesh=N0, box=100.0, a=args.a, fr0_abs=args.fr0, tol=1e-8, precision=mgfr.MIXED,
                         refine_levels=2, pre_smooth=args.smooth, post_smooth=args.smooth,
                         coarse_sweeps=4 if args.coarse_sweeps is None else args.coarse_sweeps,
                         prolong=prolong_code(args))
    amr = mgfr.Amr(params, max_blocks=262144)
    amr.set_relaxation32(args.omega)
    amr.reserve_particles(pos.shape[0])  # binned composite assignment
    for _ in range(args.warmup):
        amr.solve(pos)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        u0, st = amr.solve(pos)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    nb = [int(amr.level(l)[0].shape[0]) for l in (1, 2)]
    cells = N0 ** 3 + 512 * sum(nb)
    del amr, pos
    torch.cuda.empty_cache()
    spectra = None if args.no_fixed_compare else {"64^3+2 vs 256^3": amr_vs_fixed(args, log, 64, 256),
                                                   "128^3+2 vs 512^3": amr_vs_fixed(args, log, 128, 512)}
    log(f"[amr] step {ms:.2f} ms, blocks {nb}, cycles {[s.vcycles for s in st]}, res {[f'{s.res:.1e}' for s in st]}")
    return {
        "metric": "cells/s to converged f_R solve (res<1e-8) on the adaptive mesh (base + refined cells)",
        "value": cells / (ms * 1e-3), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"256^3 base + 2 refined levels (8^3 blocks where a cell holds > 8 particles), "
                               f"256^3 particles, Zel'dovich k^-2 rms 5 + 50 NFW halos (c 5-10), seed 4, "
                               f"a={args.a}, |f_R0|={args.fr0}; step = flagging + binned composite CIC (Sec. 3.1) + "
                               f"base and refined-level mixed solves (float64 defect loop, float32 correction "
                               f"cycles)",
                   "coarse_sweeps": params.coarse_sweeps, "omega": args.omega,
                   "blocks_per_level": nb, "cells": cells, "vcycles_per_level": [s.vcycles for s in st],
                   "res_per_level": [s.res for s in st], "power_ratio_adaptive_vs_fixed": spectra},
        "roofline": None,
    }


def amr_vs_fixed(args, log, N0=64, N=256):
    """The paper's comparison of adaptive and fixed meshes (Sec. 5.1) on a
    synthetic load: P(delta + delta_eff) / P(delta) of an N0^3 base with two
    refined levels (finest N^3 = (4 N0)^3) against the fixed N^3 mesh, N^3
    particles (Zel'dovich rms 5 + 20 Plummer halos, seed 2), |f_R0| = 1e-6 and
    1e-5, mixed solves; untimed.  With N = 512 the base's 128^3 cells hold 64
    particles each, so level 1 covers the box and level 2 refines where a
    256^3 cell holds more than 8: the finest-level structure the paper's
    64^3 base reaches with three levels."""
    import numpy as np
    import torch
    from paper_1305_2418_amd import mgfr, synth
    dev = torch.device("cuda:0")
    pos = synth.clustered_load(N, 100.0, rms=5.0, seed=2, n_halos=20, device=dev).to(dev)
    out = {}
    for fr0 in (1e-6, 1e-5):
        amr = mgfr.Amr(mgfr.Params(mesh=N0, fr0_abs=fr0, refine_levels=2, precision=mgfr.MIXED, pre_smooth=4,
                                   post_smooth=4, prolong=1, coarse_sweeps=4), max_blocks=262144)
        amr.reserve_particles(pos.shape[0])
        amr.solve(pos)
        d_a, e_a = amr.composite()
        nbl = [int(amr.level(l)[0].shape[0]) for l in (1, 2)]
        del amr
        fixed = mgfr.Solver(mgfr.Params(mesh=N, fr0_abs=fr0, precision=mgfr.MIXED, pre_smooth=4, post_smooth=4,
                                        prolong=1))
        d_f = fixed.assign_density(pos)
        u_f, _, _ = fixed.solve(d_f, want_dfr=False)
        e_f = fixed.effective_density(d_f, u_f)
        k, r_a, _, _ = fixed.power_ratio(d_a, e_a)
        _, r_f, _, _ = fixed.power_ratio(d_f, e_f)
        sel = k <= 5.0
        dev_mod = float(np.max(np.abs((r_a[sel] - 1) / (r_f[sel] - 1) - 1)))
        dev_abs = float(np.max(np.abs(r_a[sel] - r_f[sel])))
        log(f"[adaptive {N0}^3 + 2 vs fixed {N}^3, |f_R0|={fr0}] blocks {nbl}; enhancement P(d+d_eff)/P(d) - 1 at k <= 5 h/Mpc "
            f"agrees to {dev_mod:.1%} (ratios to {dev_abs:.3f})")
        step = max(1, len(k) // 16)
        out[str(fr0)] = {"k_h_per_Mpc": [float(x) for x in k[::step]], "adaptive": [float(x) for x in r_a[::step]],
                         "fixed": [float(x) for x in r_f[::step]], "blocks_per_level": nbl,
                         "max_rel_diff_of_enhancement_k_le_5": dev_mod, "max_abs_diff_of_ratio_k_le_5": dev_abs}
        del fixed, d_a, e_a, d_f, u_f, e_f
    return out


def run_sequence(args, log):
    """Chained time steps: kick-drift-kick particle-mesh steps of the 512^3 load
    from a = 0.9 to 1.0 (Zel'dovich rms 5 + 20 Plummer halos, linear-theory
    momenta), each solve starting from the previous step's u (the paper's
    warm start, Sec. 3.3 step 2).  A step = drift, assignment, mixed solve,
    particle-mesh acceleration (Newtonian + fifth force) and kicks.  The
    density of every step is also solved from u = 0, from the screened-limit
    guess and from the network (untimed in the step, reported per solve)."""
    import numpy as np
    import torch
    from paper_1305_2418_amd import mgfr, synth
    N, K = args.mesh, max(2, args.steps)
    a0, da = 0.9, 0.1 / K
    dev = torch.device("cuda:0")
    mk = lambda nn, a: mgfr.Solver(mgfr.Params(mesh=N, box=100.0, a=a, fr0_abs=args.fr0, tol=1e-8,
                                               precision=mgfr.MIXED, nn_mode=nn, pre_smooth=args.smooth,
                                               post_smooth=args.smooth, prolong=prolong_code(args)))
    chain = mk(mgfr.NN_NONE, a0)
    others = {"cold": mk(mgfr.NN_NONE, a0), "network": mk(mgfr.NN_COARSE, a0), "screened": mk(mgfr.NN_NONE, a0)}
    for s in [chain, *others.values()]:
        s.set_relaxation32(args.omega)
        s.set_inner_cycles(args.inner)
    net = mgfr.Net(seed=0, max_voxels=(N // 4) ** 3)
    net.set_params(np.load(WEIGHTS))
    others["network"].set_net(net)
    pos, mom = synth.initial_conditions(N, 100.0, rms=5.0, seed=args.seed, a=a0, n_halos=20, device=dev)
    pos, mom = pos.to(dev), mom.to(dev)
    chain.reserve_particles(pos.shape[0])
    delta = chain.assign_density(pos)
    u = chain.screened_guess(delta)
    u, _, st0 = chain.solve(delta, u=u, want_dfr=False)
    acc = chain.pm_accel(delta, u, pos)
    torch.cuda.synchronize()
    log(f"[steps] initial solve at a = {a0}: {st0.vcycles} cycles")
    out = {m: {"vcycles": [], "solve_ms": []} for m in ("previous", *others)}
    step_ms = []
    for k in range(K):
        a1 = a0 + da * (k + 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = chain.pm_step(pos, mom, acc, a1, delta, u)
        torch.cuda.synchronize()
        step_ms.append(1e3 * (time.perf_counter() - t0))
        out["previous"]["vcycles"].append(st.vcycles)
        out["previous"]["solve_ms"].append(st.t_solve_ms)
        for m, s in others.items():
            s.set_scale_factor(a1)
            g = s.screened_guess(delta) if m == "screened" else torch.zeros_like(delta)
            _, _, sto = s.solve(delta, u=g, want_dfr=False)
            out[m]["vcycles"].append(sto.vcycles)
            out[m]["solve_ms"].append(sto.t_solve_ms)
        log(f"[step {k}] a = {a1:.3f}: step {step_ms[-1]:.1f} ms; " +
            ", ".join(f"{m} {out[m]['vcycles'][-1]} cycles {out[m]['solve_ms'][-1]:.1f} ms" for m in out))
    ms = sum(step_ms) / len(step_ms)
    return {
        "metric": "cells/s of chained time steps (drift + CIC + solve to res<1e-8 from the previous step's u + "
                  "particle-mesh force + kicks)",
        "value": N ** 3 / (ms * 1e-3), "unit": "cells/s", "n_gpus": 1, "steps": K, "warmup": 0,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"{N}^3 particles and mesh, Zel'dovich k^-2 rms 5 + 20 Plummer halos (seed "
                               f"{args.seed}), linear-theory momenta at a = {a0}, {K} kick-drift-kick steps to "
                               f"a = 1, |f_R0| = {args.fr0}; mixed solves with omega = {args.omega}, up to {args.inner} "
                               f"correction cycles per float64 check; the other "
                               f"guesses solve the same density (reported, not part of the step)",
                   "step_ms": step_ms, "modes": out},
        "roofline": None,
    }


def calibrate_copy(log):
    """A plain streaming kernel of known traffic for the HBM byte counters:
    bitwise NOT of 1 GiB of int32 into a second 1 GiB buffer (reads and writes
    exactly 1 GiB; the kernel name is unique in this program)."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.bitwise_not(a, out=b)
    torch.cuda.synchronize()
    log("streamed 3 x 1 GiB through bitwise_not")
    del a, b


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "mgfr runs on one GPU; --gpus must be 1 "
                                   "(sharding over several GPUs is designed, not implemented)"}))
        sys.exit(2)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    import torch
    from paper_1305_2418_amd import synth

    if args.calibrate_copy:
        calibrate_copy(log)
    if args.workload == "sequence":
        print(json.dumps(run_sequence(args, log)), flush=True)
        return
    if args.workload == "amr":
        print(json.dumps(run_amr(args, log)), flush=True)
        return
    dev = torch.device("cuda:0")
    N = args.mesh
    t0 = time.perf_counter()
    pos = synth.clustered_load(N, 100.0, rms=5.0, seed=args.seed, n_halos=20, device=dev).to(dev)
    torch.cuda.synchronize()
    log(f"generated {N}^3 particles in {time.perf_counter() - t0:.1f}s")

    results = {}
    modes = [m for m in args.compare.split(",") if m and m != args.mode] + [args.mode]
    modes.sort(key=lambda m: m != "fp64")  # the float64 solve first: the others are compared with it
    for mode in modes:
        ref = results["fp64"].get("_dfr") if "fp64" in results else None
        results[mode] = run_mode(mode, args, pos, dev, log, dfr_ref=ref)
    results.get("fp64", {}).pop("_dfr", None)
    head = results[args.mode]
    other_a = {}
    for a in [float(x) for x in args.also_a.split(",") if x]:
        if a != args.a:
            other_a[str(a)] = {}
            for m in ("fp64", "mixed", "mixed_nn", "mixed_scr"):
                ref = other_a[str(a)].get("fp64", {}).get("_dfr")
                other_a[str(a)][m] = run_mode(m, args, pos, dev, log, a=a, dfr_ref=ref)
            other_a[str(a)]["fp64"].pop("_dfr", None)
    copy_gbs = measure_copy(dev, log)
    mfma = measure_mfma(N, dev, log)
    # dominant kernel of the headline mode: the finest-level smoothing sweep
    # algorithmic bytes of a red-black sweep: float64, read u and f, write u
    # (24 B/cell); float32 correction sweep, read e, r and u, write e (16 B/cell)
    if args.mode.startswith("fp64"):
        kernel, bpc, design_bpc = ("k_sweep_fused" if N >= 512 else "k_sweep_half (x2 per sweep)"), 24.0, 24.0
        src = KERNEL_SRC["fp64"]
    else:
        # one colour pass is half a sweep (8 B/cell of the sweep's 16); by its own
        # design it reads u and e of every cell, r of the updated half and
        # writes that half (12 B/cell)
        kernel, bpc, design_bpc = "k_mx_colour (x2 per sweep)", 8.0, 12.0
        src = KERNEL_SRC["mixed"]
    alg_bytes = bpc * N ** 3
    achieved = alg_bytes / (head["sweep_launch_ms"] * 1e-3) / 1e9
    design_GBs = design_bpc * N ** 3 / (head["sweep_launch_ms"] * 1e-3) / 1e9
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "sweep_traffic.json")
    if os.path.exists(tpath):
        tj = json.load(open(tpath))
        ent = tj.get(kernel.split(" ")[0])
        if ent and ent.get("source_hash") == source_hash(src) and ent.get("mesh") == N:
            traffic = ent.get("bytes_per_launch")
    out = {
        "metric": "cells/s to converged f_R solve (res<1e-8), plain FP64 MG vs mixed+NN warm start",
        "value": head["cells_per_s"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.mode.startswith("fp64") else "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": f"{N}^3 mesh, {N}^3 particles (float32), 100 Mpc/h, a={args.a}, |f_R0|={args.fr0}, "
                        f"Zel'dovich k^-2 rms 5 + 20 Plummer halos, seed {args.seed}; step = CIC + solve to 1e-8 with "
                        f"V({args.smooth},{args.smooth}), {args.prolong} prolongation, + fifth force; initial guess "
                        f"per mode: u = 0 (fp64, mixed), the network's prediction on the N/4 mesh (mixed_nn, its "
                        f"time included), the screened-limit guess (_scr, its time included); mixed modes: float32 "
                        f"correction sweeps relaxed by omega = {args.omega}, up to {args.inner} correction cycles per float64 "
                        f"residual check",
            "mode": args.mode,
            "modes": results,
            "modes_other_a": other_a,
        },
        "mfma": mfma,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
                     "launch_ms": head["sweep_launch_ms"], "alg_bytes_per_launch": alg_bytes,
                     "achievable_GBs": copy_gbs, "frac_of_achievable": achieved / copy_gbs,
                     "design_bytes_per_launch": design_bpc * N ** 3, "design_GBs": design_GBs,
                     "counted_GBs": traffic / (head["sweep_launch_ms"] * 1e-3) / 1e9 if traffic else None},
    }
    if not args.no_cpu_baseline:
        base, d_o, dfr_o = cpu_baseline(args, log)
        base["gpu_vcycles"] = head["vcycles"][-1]
        out["cpu_baseline"] = base
        out["config"]["mixed_vs_oracle"] = mixed_vs_oracle(args, d_o, dfr_o, dev, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
