"""Block-refined levels (one-way interface) against the dense oracle: the same
blocks are refined, every level converges in the same number of V-cycles and
the level solutions agree to 1e-10 relative (float64), 1e-6 with the
mixed-precision base solve."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1305_2418_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _compare(N0, nref, fr0, a, seed, precision, tol_rel, omega=None):
    from paper_1305_2418_amd import mgfr
    pos = synth.clustered_load(N0, 100.0, rms=5.0, seed=seed, n_halos=50, profile="nfw")
    s_o, us, ms, sts = O.amr_solve(O.params(mesh=N0, fr0_abs=fr0, a=a), nref, pos.numpy())
    assert s_o == 0
    amr = mgfr.Amr(mgfr.Params(mesh=N0, fr0_abs=fr0, a=a, refine_levels=nref, precision=precision),
                   max_blocks=20000)
    if omega is not None:
        amr.set_relaxation32(omega)
    u0, st = amr.solve(pos.to(DEV))
    assert all(s.status == 0 for s in st)
    assert np.abs(u0.cpu().numpy() - us[0]).max() <= tol_rel * max(1.0, np.abs(us[0]).max())
    for l in range(1, nref + 1):
        org, ul = amr.level(l)
        N = N0 << l
        # identical block sets
        mask = ms[l].astype(bool)
        oracle_blocks = {tuple(x) for x in np.argwhere(mask[::8, ::8, ::8]) * 8}
        assert {tuple(x) for x in org.tolist()} == oracle_blocks, f"level {l} blocks differ"
        ref = np.stack([us[l][o[0]:o[0] + 8, o[1]:o[1] + 8, o[2]:o[2] + 8] for o in org])
        err = np.abs(ul.cpu().numpy() - ref).max() / np.abs(ref).max()
        print(f"  level {l}: {len(org)} blocks, cycles {st[l].vcycles} (oracle {sts[l].vcycles}), "
              f"res {st[l].res:.2e}, rel err {err:.2e}")
        assert err < tol_rel
        if precision == mgfr.FP64:
            assert st[l].vcycles == sts[l].vcycles


@pytest.mark.parametrize("N0,nref,fr0,a,seed", [(32, 2, 1e-6, 1.0, 4), (32, 1, 1e-5, 1.0, 5), (64, 2, 1e-6, 0.7, 6)])
def test_amr_fp64_matches_oracle(N0, nref, fr0, a, seed):
    from paper_1305_2418_amd import mgfr
    print(f"[case] amr N0={N0} nref={nref} fr0={fr0} a={a}", flush=True)
    _compare(N0, nref, fr0, a, seed, mgfr.FP64, 1e-10)


def test_amr_mixed_base_matches_oracle():
    from paper_1305_2418_amd import mgfr
    print("[case] amr mixed base", flush=True)
    _compare(32, 2, 1e-6, 1.0, 4, mgfr.MIXED, 1e-6)


@pytest.mark.parametrize("omega", [1.2, 1.6])
def test_amr_mixed_relaxed_matches_oracle(omega):
    """Over-relaxed float32 correction sweeps on the base and refined levels
    change only the cycle counts: the answer is the oracle's."""
    from paper_1305_2418_amd import mgfr
    print(f"[case] amr mixed omega={omega}", flush=True)
    _compare(64, 2, 1e-6, 0.7, 6, mgfr.MIXED, 1e-6, omega=omega)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fully_refined_level_matches_uniform_oracle(precision):
    """Every base cell holds more than 8 particles: level 1 covers the whole
    periodic box, and the library's level-1 field must equal the uniform
    oracle's solve at twice the resolution."""
    from paper_1305_2418_amd import mgfr
    N0 = 32
    print(f"[case] fully refined level, {precision}", flush=True)
    pos = synth.clustered_load(128, 100.0, rms=0.3, seed=6, n_halos=0)
    idx = np.floor(pos.numpy() / (100.0 / N0)).astype(int) % N0
    cnt = np.zeros((N0,) * 3, int)
    np.add.at(cnt, (idx[:, 0], idx[:, 1], idx[:, 2]), 1)
    assert cnt.min() > 8
    prec = mgfr.FP64 if precision == "fp64" else mgfr.MIXED
    amr = mgfr.Amr(mgfr.Params(mesh=N0, fr0_abs=1e-5, refine_levels=1, precision=prec, tol=1e-10),
                   max_blocks=20000)
    u0, st = amr.solve(pos.to(DEV))
    org, ul = amr.level(1)
    assert len(org) == (2 * N0 // 8) ** 3 and all(s.status == 0 for s in st)
    d1 = O.density_contrast(O.cic_assign(2 * N0, 100.0, pos.numpy()))
    s1, u1, _, _ = O.solve(O.params(mesh=2 * N0, fr0_abs=1e-5, tol=1e-10), d1)
    ul = ul.cpu().numpy()
    full = np.empty((2 * N0,) * 3)
    for o, blk in zip(org, ul):
        full[o[0]:o[0] + 8, o[1]:o[1] + 8, o[2]:o[2] + 8] = blk
    err = np.abs(full - u1).max() / np.abs(u1).max()
    print(f"  level-1 cycles {st[1].vcycles}, rel diff from the uniform 64^3 oracle {err:.2e}")
    assert err <= 1e-8


def test_amr_rejects_bad_arguments():
    from paper_1305_2418_amd import mgfr
    with pytest.raises(mgfr.MgfrError):
        mgfr.Amr(mgfr.Params(mesh=32, refine_levels=3))
    pos = synth.clustered_load(32, 100.0, rms=5.0, seed=4, n_halos=50, profile="nfw").to(DEV)
    amr = mgfr.Amr(mgfr.Params(mesh=32, fr0_abs=1e-6, refine_levels=2), max_blocks=4)
    with pytest.raises(mgfr.MgfrError) as ei:
        amr.solve(pos)
    assert "max_blocks" in str(ei.value)


def _val_fn(u0, levels, N0):
    """value(l, i, j, k) of the library's solution on level l (0 = base), wrapped;
    None where level l has no block."""
    def val(l, i, j, k):
        N = N0 << l
        i, j, k = i % N, j % N, k % N
        if l == 0:
            return u0[i, j, k]
        idx, ul = levels[l]
        b = idx.get((i - i % 8, j - j % 8, k - k % 8))
        return None if b is None else ul[b, i % 8, j % 8, k % 8]
    return val


def _prolong_parent(val, l, i, j, k):
    """Linear reconstruction (Sec. 3.3) of the level-(l-1) solution at level-l cell (i,j,k)."""
    I, J, K = i // 2, j // 2, k // 2
    v = val(l - 1, I, J, K)
    for d, s in ((0, 1 if i % 2 else -1), (1, 1 if j % 2 else -1), (2, 1 if k % 2 else -1)):
        e = [0, 0, 0]
        e[d] = 1
        v += s * (val(l - 1, I + e[0], J + e[1], K + e[2]) - val(l - 1, I - e[0], J - e[1], K - e[2])) / 8.0
    return v


def test_config4_full_size_sampled_residual():
    """The adaptive configuration at its own size: 256^3 base plus two levels on
    256^3 particles with 50 NFW halos (seed 4), mixed precision with the
    benchmark's schedule.  The library's block sets equal the oracle's
    refinement flags exactly; at sampled cells of every level (random cells,
    cells next to ghost faces and, on the base and level 1, cells covered by
    the next level) the residual f - L(u) evaluated by the oracle -- composite
    masses from the particles (the library assigns them binned, as the
    benchmark does), the operator on the stencil, ghost values
    reconstructed from the parent level's solution -- is within the solve's
    tolerance of the level's scale."""
    from paper_1305_2418_amd import mgfr
    N0, nref, fr0 = 256, 2, 1e-6
    print("[case] adaptive 256^3 + 2 levels, 256^3 particles, sampled residuals", flush=True)
    pos = synth.clustered_load(N0, 100.0, rms=5.0, seed=4, n_halos=50, profile="nfw")
    params = mgfr.Params(mesh=N0, fr0_abs=fr0, refine_levels=nref, precision=mgfr.MIXED, pre_smooth=4,
                         post_smooth=4, prolong=mgfr.PROLONG_INJECT, coarse_sweeps=4)
    amr = mgfr.Amr(params, max_blocks=65536)
    amr.set_relaxation32(1.2)
    amr.reserve_particles(pos.shape[0])  # the benchmark's binned assignment
    u0, st = amr.solve(pos.to(DEV))
    assert all(s.status == 0 and s.res <= 1e-8 for s in st), [(s.status, s.res) for s in st]
    u0 = u0.cpu().numpy()
    pnp = pos.numpy()
    op = O.params(mesh=N0, fr0_abs=fr0)
    blk = O.amr_flags(op, nref, pnp)
    levels = {}
    for l in (1, 2):
        org, ul = amr.level(l)
        org = org.tolist()
        M = (N0 << l) // 8
        got = np.zeros((M, M, M), np.uint8)
        for o in org:
            got[o[0] // 8, o[1] // 8, o[2] // 8] = 1
        assert np.array_equal(got, blk[l]), f"level {l} block sets differ"
        levels[l] = ({tuple(o): b for b, o in enumerate(org)}, ul.cpu().numpy())
    print(f"  blocks {[len(levels[l][0]) for l in (1, 2)]}, cycles {[s.vcycles for s in st]}", flush=True)
    val = _val_fn(u0, levels, N0)
    rng = np.random.default_rng(44)
    fb, beta, C = O.background(op)
    srcs = beta * 0.3
    samples = []  # (level, i, j, k)
    for l in range(nref + 1):
        N = N0 << l
        if l == 0:
            cand = rng.integers(0, N, (600, 3))
            covered = np.argwhere(blk[1])[rng.choice(int(blk[1].sum()), 100)] * 4 + rng.integers(0, 4, (100, 3))
            cand = np.concatenate([cand, covered])
        else:
            org = np.array(list(levels[l][0].keys()))
            pick = org[rng.choice(len(org), 500)] + rng.integers(0, 8, (500, 3))
            face = org[rng.choice(len(org), 400)]
            fc = rng.integers(0, 8, (400, 3))
            ax = rng.integers(0, 3, 400)
            fc[np.arange(400), ax] = np.where(rng.random(400) < 0.5, 0, 7)  # on a block face
            cand = np.concatenate([pick, face + fc])
            if l < nref:
                org2 = np.argwhere(blk[l + 1]) * 8 // 2  # level-l cells under level-(l+1) blocks
                cand = np.concatenate([cand, org2[rng.choice(len(org2), 100)] + rng.integers(0, 4, (100, 3))])
        samples += [(l, *c) for c in cand.tolist()]
    samples = sorted(set(samples))
    # particles that can reach the sampled cells: those within one base cell of them
    h0 = 100.0 / N0
    bc = np.floor(pnp / h0).astype(np.int64) % N0
    key = (bc[:, 0] * N0 + bc[:, 1]) * N0 + bc[:, 2]
    order = np.argsort(key, kind="stable")
    ks = key[order]
    near = set()
    for (l, i, j, k) in samples:
        I, J, K = i >> l, j >> l, k >> l
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                for c in (-1, 0, 1):
                    near.add((((I + a) % N0) * N0 + (J + b) % N0) * N0 + (K + c) % N0)
    near = np.array(sorted(near), np.int64)
    lo = np.searchsorted(ks, near, "left")
    hi = np.searchsorted(ks, near, "right")
    sub = np.concatenate([order[a:b] for a, b in zip(lo, hi)])
    lev = np.array([s[0] for s in samples], np.int32)
    ijk = np.array([s[1:] for s in samples], np.int32)
    mass = O.amr_cic_cells(op, nref, blk, pnp[sub], lev, ijk)
    total = float(pnp.shape[0])
    for l in range(nref + 1):
        N = N0 << l
        sel = [t for t, s in enumerate(samples) if s[0] == l]
        uc, nb = [], []
        for t in sel:
            _, i, j, k = samples[t]
            uc.append(val(l, i, j, k))
            row = []
            for (di, dj, dk) in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                v = val(l, i + di, j + dj, k + dk)
                row.append(_prolong_parent(val, l, i + di, j + dj, k + dk) if v is None else v)
            nb.append(row)
        f = srcs * (mass[sel] / (total / N ** 3) - 1.0)
        r = f - O.op_stencil(100.0 / N, beta * C, np.array(uc), np.array(nb))
        worst = np.abs(r).max() / st[l].scale
        print(f"  level {l}: {len(sel)} cells, max |f - L(u)| / D = {worst:.2e} (solve: {st[l].res:.2e})")
        assert worst <= 1.01e-8


@pytest.mark.parametrize("fr0,binned", [(1e-6, False), (1e-5, False), (1e-6, True)])
def test_composite_spectrum_matches_oracle(fr0, binned):
    """The adaptive solution on one grid (Sec. 5.1's comparison of adaptive and
    fixed meshes): composite delta and effective density of the library against
    the oracle's composite cell by cell, and the ratio P(delta + delta_eff) /
    P(delta) of the library's shell spectra against numpy's."""
    from paper_1305_2418_amd import mgfr
    N0, nref = 32, 2
    print(f"[case] composite spectrum fr0={fr0} binned={binned}", flush=True)
    pos = synth.clustered_load(N0, 100.0, rms=5.0, seed=4, n_halos=50, profile="nfw")
    p = O.params(mesh=N0, fr0_abs=fr0)
    s_o, blk, ds, us, ms, sts = O.amr_levels(p, nref, pos.numpy())
    assert s_o == 0
    d_o, e_o = O.amr_composite(p, ds, us, ms)
    amr = mgfr.Amr(mgfr.Params(mesh=N0, fr0_abs=fr0, refine_levels=nref), max_blocks=20000)
    if binned:
        amr.reserve_particles(pos.shape[0])
    amr.solve(pos.to(DEV))
    d, e = amr.composite()
    d, e = d.cpu().numpy(), e.cpu().numpy()
    assert np.abs(d - d_o).max() <= 1e-12 * np.abs(d_o).max()
    assert np.abs(e - e_o).max() <= 1e-9 * np.abs(d_o).max()
    Nf = N0 << nref
    k_o, r_o, pd_o, c_o = O.power_ratio(100.0, d_o, e_o, Nf // 2)
    ctx = mgfr.Solver(mgfr.Params(mesh=Nf))
    k, r, pd, c = ctx.power_ratio(torch.tensor(d, device=DEV), torch.tensor(e, device=DEV))
    print(f"  ratio at k_1 {r[0]:.4f}, k_8 {r[7]:.4f}, k_32 {r[31]:.4f}")
    assert np.array_equal(c, c_o)
    assert np.allclose(r, r_o, rtol=1e-8) and np.allclose(pd, pd_o, rtol=1e-9)


@pytest.mark.parametrize("N0,nref,npart", [(256, 2, 256), (64, 2, 96), (32, 1, 40)])
def test_binned_assignment_equals_per_particle(N0, nref, npart):
    """The binned composite assignment (particles sorted by the group of cells
    they deposit into, one LDS window per run; cubes across levels on the
    per-particle path) against the per-particle one on the same solve: the
    same composite density up to the order of the float64 sums, and the same
    converged solution up to the solve's tolerance.  Covers the 256^3 configuration (256^3 particles, 50
    NFW halos) and particle counts that leave a ragged last chunk."""
    from paper_1305_2418_amd import mgfr
    print(f"[case] binned vs per-particle N0={N0} nref={nref} np={npart}^3", flush=True)
    pos = synth.clustered_load(npart, 100.0, rms=5.0, seed=4, n_halos=50, profile="nfw").to(DEV)
    out = []
    for binned in (False, True):
        amr = mgfr.Amr(mgfr.Params(mesh=N0, fr0_abs=1e-6, refine_levels=nref), max_blocks=65536)
        if binned:
            amr.reserve_particles(pos.shape[0] + 5)
        u0, st = amr.solve(pos)
        assert all(s.status == 0 for s in st)
        d, _ = amr.composite()
        out.append((d.cpu().numpy(), u0.cpu().numpy()))
        del amr
    (d0, u0), (d1, u1) = out
    assert np.abs(d1 - d0).max() <= 1e-12 * np.abs(d0).max()
    # both solves stop at residual 1e-8: their answers differ by less than that error
    assert np.abs(u1 - u0).max() <= 1e-6 * np.abs(u0).max()
