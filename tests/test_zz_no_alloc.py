"""The allocation-free assignment (mgfr_assign_density_noalloc) against the
context-based mgfr_assign_density on the same particles: two calls in a row,
the second on a smaller mesh with fewer particles, with and without masses.
Both sides are float64 sums of the same cloud-in-cell weights; only the order
of the atomic additions differs, so they agree to a few ulps of the cell
mass."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1305_2418_amd import mgfr, synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _reference(pos, mesh, box, mass, binning):
    s = mgfr.Solver(mgfr.Params(mesh=mesh, box=box), binning=binning)
    try:
        d = s.assign_density(pos, mass)
        torch.cuda.synchronize()
        return d.clone()
    finally:
        s.close()


def _case(mesh, npart_side, box, seed, with_mass):
    pos = synth.clustered_load(npart_side, box, rms=1.0, seed=seed).to("cuda:0")
    mass = None
    if with_mass:
        g = np.random.default_rng(seed + 7)
        mass = torch.from_numpy(g.uniform(0.5, 1.5, pos.shape[0])).to("cuda:0")
    return pos, mass


def test_noalloc_matches_context_assignment_twice_smaller_second():
    print("noalloc: 64^3 mesh, 64^3 particles, then 32^3 mesh, 24^3 particles", flush=True)
    cases = [(64, 64, 100.0, 11, False), (32, 24, 80.0, 12, True)]
    outs = []
    for mesh, nps, box, seed, wm in cases:
        pos, mass = _case(mesh, nps, box, seed, wm)
        got = mgfr.assign_density_noalloc(pos, mesh, box, mass)
        torch.cuda.synchronize()
        got = got.clone()
        for binning in (False, True):
            ref = _reference(pos, mesh, box, mass, binning)
            err = (got - ref).abs().max().item()
            assert err <= TOL * max(1.0, ref.abs().max().item()), (mesh, binning, err)
        assert abs(got.sum().item()) < 1e-9 * got.numel()
        outs.append(got)
    assert outs[1].shape == (32, 32, 32)


def test_noalloc_into_preallocated_output_and_errors():
    pos, _ = _case(16, 16, 50.0, 3, False)
    out = torch.full((16, 16, 16), 7.0, dtype=torch.float64, device="cuda:0")
    mgfr.assign_density_noalloc(pos, 16, 50.0, out=out)
    ref = _reference(pos, 16, 50.0, None, False)
    torch.cuda.synchronize()
    assert (out - ref).abs().max().item() <= TOL * max(1.0, ref.abs().max().item())
    lib = mgfr.lib()
    # host-side argument checks: nothing is launched for these
    bad = [(24, 50.0, b"power of two"), (2048, 50.0, b"maximum"), (16, -1.0, b"box")]
    for mesh, box, words in bad:
        rc = lib.mgfr_assign_density_noalloc(mesh, box, None, ctypes.c_void_p(pos.data_ptr()), None,
                                             pos.shape[0], ctypes.c_void_p(out.data_ptr()))
        assert rc == mgfr.MGFR_ERR_ARG, (mesh, box, rc)
        assert words in lib.mgfr_last_error(), lib.mgfr_last_error()
    # a non-finite position is reported, not written past the mesh
    p2 = pos.clone()
    p2[5, 1] = float("nan")
    with pytest.raises(mgfr.MgfrError) as ei:
        mgfr.assign_density_noalloc(p2, 16, 50.0, out=out)
    assert ei.value.code == mgfr.MGFR_ERR_NONFINITE
    # and the next good call is clean again (the flag is reset per call)
    mgfr.assign_density_noalloc(pos, 16, 50.0, out=out)
    torch.cuda.synchronize()
    assert (out - ref).abs().max().item() <= TOL * max(1.0, ref.abs().max().item())
