"""Host-side logic of bench.py: the roofline arithmetic of the binning and
list-build kernels, and the one-GPU contract.  No GPU is used."""

import importlib.util
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_build_rooflines_arithmetic():
    b = _bench()
    n, n_cells, mean_list = 1000, 40, 75.0
    # 25 rebuilds: binning 2 ms in all (80 us each), list build 50 ms (2 ms each)
    tm = {"force": (10.0, 100), "binning": (2.0, 25), "neighbor": (50.0, 25)}
    cand = 19.5
    r = b._build_rooflines(tm, n, mean_list, n_cells, cand)
    assert r["binning"]["avg_call_us"] == pytest.approx(80.0)
    assert r["binning"]["alg_bytes_per_call"] == pytest.approx(132.0 * n)
    assert r["binning"]["achieved"] == pytest.approx(132.0 * n / 80e-6 / 1e9)
    assert r["binning"]["frac"] == pytest.approx(r["binning"]["achieved"] / 8000.0)
    nb = r["neighbor"]
    assert nb["bound"] == "alu" and nb["unit"] == "T FP64 instr/s"
    assert nb["candidates_per_atom"] == cand
    assert nb["cell_stencil_candidates_per_atom"] == pytest.approx(27.0 * n / n_cells)
    assert nb["achieved"] == pytest.approx(8.0 * cand * n / 2e-3 / 1e12)
    # unfused FP64 instructions issue at 256 CUs x 64 lanes x 2.4 GHz = 39.32 T/s
    assert nb["peak"] == pytest.approx(39.3216)
    assert nb["frac"] == pytest.approx(nb["achieved"] / 39.3216)
    assert nb["alg_bytes_per_call"] == pytest.approx((28.0 + 4.0 * mean_list) * n)
    assert nb["hbm_frac"] == pytest.approx(nb["hbm_achieved_gbs"] / 8000.0)


def test_trimmed_stencil_against_sampling_and_limits():
    """Subcells of the 5^3 stencil that the cutoff sphere reaches: every one
    while the farthest offset's nearest corner lies within rl (side <
    rl / sqrt(3)), the same mean as random sampling of the atom's place
    (an independent estimate), fewer as cells grow."""
    b = _bench()
    assert b._trimmed_subcells(0.5) == 125.0
    rng = np.random.default_rng(7)
    for ratio in (1.0, 1.3):
        h = 0.5 * ratio
        p = rng.random((40000, 3)) * h
        off = np.array([-2, -1, 0, 1, 2])

        def gap(q, d):  # distance from q (in [0, h)) to the subcell at offset d
            return np.where(d > 0, d * h - q, np.where(d < 0, q + (-d - 1) * h, 0.0))

        gx, gy, gz = (gap(p[:, a, None], off[None, :]) ** 2 for a in range(3))
        hits = (gx[:, :, None, None] + gy[:, None, :, None] + gz[:, None, None, :] < 1.0).sum((1, 2, 3))
        assert b._trimmed_subcells(ratio) == pytest.approx(hits.mean(), rel=0.01)
    assert b._trimmed_subcells(1.0) > b._trimmed_subcells(1.3) > b._trimmed_subcells(2.0)
    # whole boxes: a box too small for the trimmed walk counts the full stencil
    L = 2.8 * 3.2  # 3 cells per axis < block edge 2 + 2
    assert b.stencil_candidates([(270, L)]) == pytest.approx(270 / (8 * 27) * 125)


def test_force_flops_arithmetic():
    b = _bench()
    r = b._force_flops(1000, 75.0, 1e-3)
    n_int = 75.0 * (2.5 / 2.8) ** 3
    assert r["fp64_flops_per_launch"] == pytest.approx((8 * 75.0 + 15 * n_int) * 1000)
    assert r["fp64_tflops"] == pytest.approx(r["fp64_flops_per_launch"] / 1e-3 / 1e12)
    assert r["fp64_frac"] == pytest.approx(r["fp64_tflops"] / 78.6)


def test_force_roofline_counts_the_force_sum_bytes():
    b = _bench()
    r = b._force_roofline(1000, 75.0, 1e-3, traffic=4.0e5)
    # count 4 + list 4 n + x_i 24 + F_i 24 per atom; the fused kernel's own
    # 100 + 4 n beside it
    assert r["alg_bytes_per_atom"] == pytest.approx(352.0)
    assert r["achieved"] == pytest.approx(352.0 * 1000 / 1e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["fused_kernel"]["bytes_per_atom"] == pytest.approx(400.0)
    assert r["traffic_frac"] == pytest.approx(4.0e5 / 1e-3 / 1e9 / 8000.0)


def test_build_rooflines_skip_kernels_not_run():
    b = _bench()
    assert b._build_rooflines({"force": (1.0, 10), "neighbor": (0.0, 0)}, 10, 1.0, 1, 5.0) == {}


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    out = json.loads(p.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]
