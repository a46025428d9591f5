"""Host-side logic that runs without a GPU: the ctypes mirrors of the C
structs against the header, the benchmark's argument handling, the rocprof
summary arithmetic and the seeded synthetic loads."""
import json
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "mgfr.h")


def _struct_fields(name):
    """Field names of `typedef struct name {...} name;` in the public header, in order."""
    txt = open(HDR).read()
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), txt, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        # "double box", "int n", "double res_hist[MGFR_MAX_HIST]"
        m = re.match(r"(?:const\s+)?\w+\s+\**(\w+)", decl)
        fields.append(m.group(1))
    return fields


def test_ctypes_structs_mirror_the_header():
    from paper_1305_2418_amd import mgfr
    assert [f for f, _ in mgfr._Params._fields_] == _struct_fields("mgfr_params")
    assert [f for f, _ in mgfr._Stats._fields_] == _struct_fields("mgfr_stats")
    # the dataclass passes its fields to the C struct in the header's order
    p = mgfr.Params(mesh=64, a=0.5, fr0_abs=3e-6, pre_smooth=4, prolong=1, precision=1, nn_mode=1,
                    max_du=1.5, coarse_cycles=2)
    c = p.to_c()
    for f, _ in mgfr._Params._fields_:
        assert getattr(c, f) == pytest.approx(getattr(p, f)), f


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_summary_scales_by_the_streaming_kernel(tmp_path):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) are scaled by what they read
    for the 1 GiB streaming kernel; the largest dispatch of a kernel is taken,
    matched by its exact name (not k_mx_colour_zero for k_mx_colour); the
    record carries the source hash the benchmark checks before using it."""
    from paper_1305_2418_amd import profile_summary as ps
    fdir, wdir = tmp_path / "f", tmp_path / "w"
    fdir.mkdir()
    wdir.mkdir()
    hdr = "Kernel_Name,Counter_Name,Counter_Value\n"
    (fdir / "x_counter_collection.csv").write_text(
        hdr + "void at::native::bitwise_not_kernel(...),FETCH_SIZE,524288\n"
        "k_mx_colour(ColourArgs),FETCH_SIZE,1000\nk_mx_colour(ColourArgs),FETCH_SIZE,800000\n"
        "mgfr::(anonymous namespace)::k_mx_colour_zero(ColourArgs),FETCH_SIZE,900000\n")
    (wdir / "x_counter_collection.csv").write_text(
        hdr + "void at::native::bitwise_not_kernel(...),WRITE_SIZE,1048576\nk_mx_colour(ColourArgs),WRITE_SIZE,262144\n")
    out = tmp_path / "t.json"
    ps.traffic(str(fdir), str(wdir), 512, str(out))
    t = json.load(open(out))
    assert t["calibration"]["copy_bytes"] == 1 << 30
    e = t["k_mx_colour"]
    assert e["fetch_scale"] == pytest.approx(2.0) and e["write_scale"] == pytest.approx(1.0)
    assert e["bytes_per_launch"] == pytest.approx((800000 * 2.0 + 262144 * 1.0) * 1024)
    assert e["mesh"] == 512 and len(e["source_hash"]) == 16
    sys.path.insert(0, ROOT)
    import bench
    assert e["source_hash"] == bench.source_hash(bench.KERNEL_SRC["mixed"])


def test_synthetic_loads_are_seeded_and_in_the_box():
    from paper_1305_2418_amd import synth
    a = synth.clustered_load(16, 100.0, rms=5.0, seed=7, n_halos=3).numpy()
    b = synth.clustered_load(16, 100.0, rms=5.0, seed=7, n_halos=3).numpy()
    c = synth.clustered_load(16, 100.0, rms=5.0, seed=8, n_halos=3).numpy()
    assert a.shape == (16 ** 3, 3) and a.dtype == np.float32
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.min() >= 0.0 and a.max() < 100.0
    # halos relocate particles: the load is clustered (some cell holds many particles)
    cells = np.floor(a / (100.0 / 16)).astype(int)
    counts = np.bincount((cells[:, 0] * 16 + cells[:, 1]) * 16 + cells[:, 2], minlength=16 ** 3)
    assert counts.sum() == 16 ** 3 and counts.max() > 20
