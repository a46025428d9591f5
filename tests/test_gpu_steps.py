"""Chained time steps (the solve of each step starts from the previous step's
u, Sec. 3.3 step 2) against the oracle: the particle-mesh acceleration, the
kick-drift update, and whole kick-drift-kick steps.  Each step of the
library's chain is repeated by the oracle from the library's state at the
start of that step, so every comparison covers one step's rounding:

* positions: bit for bit (the drift uses the same float32 inputs and one
  float64 fused multiply-add on both sides);
* u: the oracle's number of V-cycles from the same guess, 1e-10 relative;
* accelerations: float32 rounding (the output type) over a float64 floor;
* momenta: the float32 rounding of the last half kick.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1305_2418_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _mg():
    from paper_1305_2418_amd import mgfr
    return mgfr


def _acc_close(a, ref):
    a = np.asarray(a, np.float64)
    scale = np.abs(ref).max()
    return np.all(np.abs(a - ref) <= 6e-8 * np.abs(ref) + 1e-10 * scale)


@pytest.mark.parametrize("with_field", [False, True])
def test_pm_accel_matches_oracle(with_field):
    mg = _mg()
    N = 64
    print(f"[case] pm accel N={N} field={with_field}", flush=True)
    pos = synth.clustered_load(N, 100.0, rms=5.0, seed=41, n_halos=10)
    p = O.params(mesh=N, a=0.7, fr0_abs=1e-5)
    d = O.density_contrast(O.cic_assign(N, 100.0, pos.numpy()))
    u = O.solve(p, d, want_dfr=False)[1] if with_field else None
    ref = O.pm_accel(p, d, u, pos.numpy())
    s = mg.Solver(mg.Params(mesh=N, a=0.7, fr0_abs=1e-5))
    g = s.pm_accel(torch.tensor(d, device=DEV), None if u is None else torch.tensor(u, device=DEV), pos.to(DEV))
    assert _acc_close(g.cpu().numpy(), ref)
    # momentum: exact for the Newtonian part
    if not with_field:
        gs = g.double().sum(0).abs().max().item()
        assert gs <= 1e-5 * g.double().abs().sum(0).max().item()


def test_kick_drift_is_bitwise_the_oracle():
    mg = _mg()
    rng = np.random.default_rng(2)
    n = 10007
    pos = rng.uniform(-5, 105, (n, 3)).astype(np.float32)
    mom = rng.normal(0, 300, (n, 3)).astype(np.float32)
    acc = rng.normal(0, 2e4, (n, 3)).astype(np.float32)
    s = mg.Solver(mg.Params(mesh=16))
    for kick, drift, use_acc in ((3.1e-3, 1.7e-3, True), (0.0, 2.2e-3, False), (1.3e-3, 0.0, True)):
        pg, mgm = torch.tensor(pos, device=DEV), torch.tensor(mom, device=DEV)
        s.kick_drift(pg, mgm, torch.tensor(acc, device=DEV) if use_acc else None, kick, drift)
        po, mo = pos.copy(), mom.copy()
        O.kick_drift(po, mo, acc if use_acc else None, kick, drift, 100.0)
        assert np.array_equal(pg.cpu().numpy(), po) and np.array_equal(mgm.cpu().numpy(), mo)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_timed"])
def test_pm_steps_match_oracle_step_by_step(precision):
    """Three kick-drift-kick steps a = 0.80 -> 0.95 of 64^3 particles (Zel'dovich
    rms 5 + 20 Plummer halos, linear-theory momenta) on the 64^3 mesh at
    |f_R0| = 1e-5.  FP64: the oracle's schedule, 1e-10; mixed (also with the
    step-chain benchmark's omega = 1.2 and three correction cycles per float64
    check): the oracle's converged solution from the same guess, 1e-6 (and
    each solve from the previous step's u takes fewer V-cycles than from
    u = 0)."""
    mg = _mg()
    N, fr0 = 64, 1e-5
    print(f"[case] pm steps {precision}", flush=True)
    pos_c, mom_c = synth.initial_conditions(N, 100.0, rms=5.0, seed=3, a=0.8, n_halos=20)
    prec = mg.FP64 if precision == "fp64" else mg.MIXED
    s = mg.Solver(mg.Params(mesh=N, a=0.8, fr0_abs=fr0, precision=prec, max_vcycles=80))
    if precision == "mixed_timed":
        s.set_relaxation32(1.2)
        s.set_inner_cycles(3)
    pos, mom = pos_c.to(DEV), mom_c.to(DEV)
    delta = s.assign_density(pos)
    u, _, _ = s.solve(delta, want_dfr=False)
    acc = s.pm_accel(delta, u, pos)
    a = 0.8
    for step in range(3):
        a1 = a + 0.05
        # the state at the start of the step, for the oracle
        x0, p0, g0, u0 = (pos.cpu().numpy().copy(), mom.cpu().numpy().copy(), acc.cpu().numpy().copy(),
                          u.cpu().numpy().copy())
        st = s.pm_step(pos, mom, acc, a1, delta, u)
        assert st.status == 0
        op = O.params(mesh=N, a=a, fr0_abs=fr0, max_vcycles=80, tol=1e-8 if precision == "fp64" else 1e-11)
        d_o, u_o, g_o, st_o = O.pm_step(op, x0, p0, g0, a1, u0)
        cold = O.solve(O.params(mesh=N, a=a1, fr0_abs=fr0, max_vcycles=80), d_o, want_dfr=False)[3].vcycles
        print(f"  step {step}: a -> {a1:.2f}, cycles {st.vcycles} (oracle {st_o.vcycles}, oracle from u = 0 {cold})",
              flush=True)
        assert np.array_equal(pos.cpu().numpy(), x0)  # x0 now holds the oracle's new positions
        assert np.abs(delta.cpu().numpy() - d_o).max() <= 1e-12 * max(1.0, np.abs(d_o).max())
        uu = u.cpu().numpy()
        if precision == "fp64":
            assert st.vcycles == st_o.vcycles
            err = np.abs(uu - u_o).max() / np.abs(u_o).max()
            assert err < 1e-10, err
            assert _acc_close(acc.cpu().numpy(), g_o.astype(np.float64))
            # momenta: the last half kick rounds |acc K2| to float32
            dm = np.abs(mom.cpu().numpy().astype(np.float64) - p0)
            assert np.all(dm <= 2.0 ** -22 * (np.abs(p0) + 1.0))
        else:
            dfr = np.expm1(uu) - np.expm1(u_o)
            err = np.abs(dfr).max() / np.abs(np.expm1(u_o)).max()
            assert err < 1e-6, err
        assert st.vcycles < cold
        # continue the library's chain from its own state
        a = a1
