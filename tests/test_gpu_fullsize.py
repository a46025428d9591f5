"""Full-size checks in the launch configuration the benchmark times.

The 512^3 workload (512^3 float32 particles, 512^3 mesh) is solved exactly as
bench.py solves it; the oracle cannot solve it in seconds, so it checks
sampled outputs one by one: the CIC mass of sampled cells (a full scan of all
particles), the residual f - L(u) at sampled cells (must be within the
tolerance), delta f_R at sampled cells, and the force at sampled particles;
and the mixed solves (network warm start, screened-limit guess) must agree
with the float64 solve.  A 1024^3 mesh (the
largest the library accepts) is solved from a synthetic multi-sphere field
and checked the same way, and a 256^3 particle load is assigned to it and
its force gathered (the binning's largest tile count)."""
import math
import os

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1305_2418_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_1305_2418_amd", "weights", "unet_warmstart.npy")


@pytest.mark.timeout(600)
def test_512_workload_sampled_against_oracle():
    from paper_1305_2418_amd import mgfr
    N, a, fr0, sm, pro = 512, 1.0, 1e-6, 4, 1  # V(4,4) with injected corrections, as timed
    print("[case] 512^3 workload", flush=True)
    pos = synth.clustered_load(N, 100.0, rms=5.0, seed=3, n_halos=20, device=DEV)
    mode = mgfr.NN_COARSE if os.path.exists(WEIGHTS) else mgfr.NN_NONE
    s = mgfr.Solver(mgfr.Params(mesh=N, a=a, fr0_abs=fr0, precision=mgfr.MIXED, nn_mode=mode,
                                pre_smooth=sm, post_smooth=sm, prolong=pro))
    s.set_relaxation32(1.2)  # as timed
    s.set_inner_cycles(3)
    net = None
    if mode == mgfr.NN_COARSE:
        net = mgfr.Net(seed=0, max_voxels=(N // 4) ** 3)
        net.set_params(np.load(WEIGHTS))
        s.set_net(net)
    delta = s.assign_density(pos)
    u, dfr, st = s.solve(delta)
    acc = s.fifth_force(u, pos)
    assert st.status == 0 and st.res <= 1e-8 and st.fell_back == 0
    print(f"  mixed{'+nn' if net else ''}: {st.vcycles} cycles, res {st.res:.2e}", flush=True)
    s64 = mgfr.Solver(mgfr.Params(mesh=N, a=a, fr0_abs=fr0, pre_smooth=sm, post_smooth=sm, prolong=pro))
    u64, dfr64, st64 = s64.solve(delta)
    assert st64.status == 0
    rel = (torch.abs(dfr - dfr64).max() / torch.abs(dfr64).max()).item()
    print(f"  fp64: {st64.vcycles} cycles; mixed vs fp64 rel dfr {rel:.2e}", flush=True)
    assert rel < 1e-6
    del s64, u64
    # mixed solve from the screened-limit guess (the bench's mixed_scr mode)
    s2 = mgfr.Solver(mgfr.Params(mesh=N, a=a, fr0_abs=fr0, precision=mgfr.MIXED, pre_smooth=sm, post_smooth=sm,
                                 prolong=pro))
    s2.set_relaxation32(1.2)
    s2.set_inner_cycles(3)
    u2, dfr2, st2 = s2.solve(delta, u=s2.screened_guess(delta))
    assert st2.status == 0 and st2.res <= 1e-8 and st2.fell_back == 0
    rel2 = (torch.abs(dfr2 - dfr64).max() / torch.abs(dfr64).max()).item()
    print(f"  mixed from the screened guess: {st2.vcycles} cycles; vs fp64 rel dfr {rel2:.2e}", flush=True)
    assert rel2 < 1e-6
    u2_h = u2.cpu().numpy()
    del s2, u2, dfr2, dfr64
    # host copies for the oracle
    pos_h = pos.cpu().numpy()
    d_h = delta.cpu().numpy()
    u_h = u.cpu().numpy()
    rng = np.random.default_rng(0)
    # 1) CIC: sampled cells (densest cells included) from a full particle scan
    flat = d_h.reshape(-1)
    cells = np.concatenate([rng.choice(N ** 3, 60, replace=False), np.argsort(flat)[-4:]]).astype(np.int64)
    mcell = O.cic_cells(N, 100.0, pos_h, cells)
    mbar = pos_h.shape[0] / N ** 3
    assert np.allclose(flat[cells], mcell / mbar - 1.0, rtol=1e-12, atol=1e-12)
    assert abs(flat.mean()) < 1e-12
    # 2) residual at sampled cells, normalised by D = max|f|
    fb, beta, C = O.background(O.params(mesh=N, a=a, fr0_abs=fr0))
    f = beta * 0.3 / a ** 3 * d_h
    D = np.abs(f).max()
    cells = np.concatenate([rng.choice(N ** 3, 200000, replace=False), np.argsort(flat)[-1000:]]).astype(np.int64)
    r = O.residual_at(u_h, f, 100.0 / N, beta * C, cells)
    print(f"  sampled max residual {np.abs(r).max() / D:.2e} (reported {st.res:.2e})", flush=True)
    assert np.abs(r).max() / D <= 1e-8
    r2 = O.residual_at(u2_h, f, 100.0 / N, beta * C, cells)
    print(f"  screened-guess solve: sampled max residual {np.abs(r2).max() / D:.2e} (reported {st2.res:.2e})",
          flush=True)
    assert np.abs(r2).max() / D <= 1e-8
    # 3) delta f_R at sampled cells
    dfr_h = dfr.cpu().numpy().reshape(-1)
    assert np.allclose(dfr_h[cells], -fb * np.expm1(u_h.reshape(-1)[cells]), rtol=1e-14, atol=1e-20)
    # 4) fifth force at sampled particles
    pidx = rng.choice(pos_h.shape[0], 3000, replace=False)
    ref = O.fifth_force_at(O.params(mesh=N, a=a, fr0_abs=fr0), u_h, pos_h[pidx])
    got = acc.cpu().numpy()[pidx].astype(np.float64)
    assert np.all(np.abs(got - ref) <= 6e-8 * np.abs(ref) + 1e-10 * np.abs(ref).max())


@pytest.mark.timeout(900)
def test_largest_mesh_1024():
    from paper_1305_2418_amd import mgfr
    N = 1024
    print("[case] 1024^3 mixed solve", flush=True)
    d = synth.spheres_delta(N, 200.0, 12, seed=5, device=DEV)
    s = mgfr.Solver(mgfr.Params(mesh=N, box=200.0, a=1.0, fr0_abs=1e-6, precision=mgfr.MIXED,
                                pre_smooth=3, post_smooth=3))
    u, dfr, st = s.solve(d)
    print(f"  {st.vcycles} cycles, res {st.res:.2e}, {st.t_solve_ms:.0f} ms", flush=True)
    assert st.status == 0 and st.res <= 1e-8
    fb, beta, C = O.background(O.params(mesh=N, box=200.0, a=1.0, fr0_abs=1e-6))
    d_h = d.cpu().numpy()
    u_h = u.cpu().numpy()
    f = beta * 0.3 * d_h
    rng = np.random.default_rng(1)
    flat = d_h.reshape(-1)
    cells = np.concatenate([rng.choice(N ** 3, 100000, replace=False), np.argsort(flat)[-500:]]).astype(np.int64)
    r = O.residual_at(u_h, f, 200.0 / N, beta * C, cells)
    assert np.abs(r).max() / np.abs(f).max() <= 1e-8
    # binned particles on the largest mesh: 2^21 tiles, eight replica counters
    # per tile, mostly sparse work units (a 256^3 load: eight particles per tile)
    print("[case] 1024^3 binned assignment and force", flush=True)
    pos = synth.clustered_load(256, 200.0, rms=5.0, seed=6, n_halos=10, device=DEV)
    delta = s.assign_density(pos)
    acc = s.fifth_force(u, pos)
    pos_h = pos.cpu().numpy()
    dflat = delta.cpu().numpy().reshape(-1)
    cells = np.concatenate([rng.choice(N ** 3, 40, replace=False), np.argsort(dflat)[-4:]]).astype(np.int64)
    mcell = O.cic_cells(N, 200.0, pos_h, cells)
    mbar = pos_h.shape[0] / N ** 3
    assert np.allclose(dflat[cells], mcell / mbar - 1.0, rtol=1e-12, atol=1e-12)
    pidx = rng.choice(pos_h.shape[0], 2000, replace=False)
    ref = O.fifth_force_at(O.params(mesh=N, box=200.0, a=1.0, fr0_abs=1e-6), u_h, pos_h[pidx])
    got = acc.cpu().numpy()[pidx].astype(np.float64)
    assert np.all(np.abs(got - ref) <= 6e-8 * np.abs(ref) + 1e-10 * np.abs(ref).max())


def test_mesh_limits_rejected():
    from paper_1305_2418_amd import mgfr
    for bad in (4, 2048, 96):
        with pytest.raises(mgfr.MgfrError):
            mgfr.Solver(mgfr.Params(mesh=bad))
